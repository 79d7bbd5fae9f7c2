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
  const int32_t *gmap, *nbr_row, *perm, *iperm, *mslot;
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
  int32_t nb, nmslot;
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
// Small fronts: one workgroup per (front, system), whole panel in LDS.
// Assembly, partial LDL^T of the pivot columns, Schur update of the u x u
// block straight into the front's update slot, panel write-back.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void k_front_small(KArgs a, const int32_t* fronts) {
  typedef typename Cx<R>::T C;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* F = reinterpret_cast<C*>(smem_raw);
  const int s = blockIdx.y;
  const int f = fronts[blockIdx.x];
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
  // X = L11^-1 (unit lower), one column per thread, into the multiplier scratch
  C* X = (C*)a.mscr + ((int64_t)s * a.nmslot + a.mslot[f]) * NB * NB;
  for (int j = threadIdx.x; j < nb; j += kThreads) {
    for (int i = 0; i < nb; ++i) {
      C v = czero<C>();
      if (i == j) {
        v.x = 1;
      } else if (i > j) {
        for (int k = j; k < i; ++k) v = cfms(v, B[k * NB + i], X[j * NB + k]);
      }
      X[j * NB + i] = v;
    }
  }
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
// Solves.  y holds the working vector in elimination order ([sys][rhs][N]);
// wv holds each front's update vector ([sys][rhs][sum u]).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool done(const int* flag) { return flag && *(volatile const int*)flag; }

// y[pos] = (S[n] if scale) * src[n], n = perm[pos]
template <typename R>
__global__ void k_gather(KArgs a, const double2* src, void* y, int nrhs, int scale, const int* flag) {
  typedef typename Cx<R>::T C;
  if (done(flag)) return;
  const int col = blockIdx.y;  // s*nrhs + r
  const int s = col / nrhs;
  C* dst = (C*)y + (int64_t)col * a.N;
  const double2* in = src + (int64_t)col * a.N;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < a.N;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int n = a.perm[q];
    double2 v = in[n];
    if (scale) v = dmul(v, sym_scale(a, s, n));
    dst[q] = from_d2<C>(v);
  }
}

// out[n] (+)= (S[n] if scale) * y[iperm[n]]
template <typename R>
__global__ void k_scatter(KArgs a, const void* y, double2* out, int nrhs, int accumulate, int scale,
                          const int* flag) {
  typedef typename Cx<R>::T C;
  if (done(flag)) return;
  const int col = blockIdx.y;
  const int s = col / nrhs;
  const C* src = (const C*)y + (int64_t)col * a.N;
  double2* o = out + (int64_t)col * a.N;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
       n += (int64_t)gridDim.x * blockDim.x) {
    double2 v = to_d2(src[a.iperm[n]]);
    if (scale) v = dmul(v, sym_scale(a, s, (int)n));
    o[n] = accumulate ? dadd(o[n], v) : v;
  }
}

template <typename C> __device__ __forceinline__ C shfl_c(C v, int lane) {
  v.x = __shfl(v.x, lane);
  v.y = __shfl(v.y, lane);
  return v;
}

// Forward sweep over one level: V = [y_p; 0] + children's update vectors,
// V <- L^-1 V over the pivot columns (in 64-column blocks: one wave solves the
// triangle, all threads apply the rectangle below it), then y_p = D^-1 V_p and
// the front's update vector = V_u.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_fwd(KArgs a, const int32_t* fronts, void* y, void* wv,
                                                   int nrhs, const int* flag) {
  typedef typename Cx<R>::T C;
  if (done(flag)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* V = reinterpret_cast<C*>(smem_raw);
  const int s = blockIdx.y;
  const int f = fronts[blockIdx.x];
  const int p = a.npiv[f], u = a.nupd[f], m = p + u;
  const int pb = a.pbeg[f];
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* Y = (C*)y + (int64_t)s * nrhs * a.N;
  C* W = (C*)wv + (int64_t)s * nrhs * a.sum_u;
  const int cb = a.child_ptr[f], ce = a.child_ptr[f + 1];
  const int32_t* g = a.gmap + a.gmap_ptr[f];
  for (int idx = threadIdx.x; idx < m * nrhs; idx += kThreads) {
    const int col = idx / m, r = idx - col * m;
    C v = r < p ? Y[(int64_t)col * a.N + pb + r] : czero<C>();
    for (int k = cb; k < ce; ++k) {
      const int gr = g[(k - cb) * m + r];
      if (gr >= 0) v = cadd(v, W[(int64_t)col * a.sum_u + a.upd_ptr[a.child_list[k]] + gr]);
    }
    V[col * m + r] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k0 = 0; k0 < p; k0 += 64) {
    const int k1 = min(k0 + 64, p), kn = k1 - k0;
    if (wave == 0) {
      for (int col = 0; col < nrhs; ++col) {
        C v = lane < kn ? V[col * m + k0 + lane] : czero<C>();
        for (int k = 0; k < kn; ++k) {
          const C vk = shfl_c(v, k);
          if (lane > k && lane < kn) v = cfms(v, L[(int64_t)(k0 + k) * m + k0 + lane], vk);
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

// Backward sweep over one level: X = [z_p; x(update rows)], then for 64-column
// blocks from the last: X_blk -= L(rows below blk, blk)^T X(below), and one
// wave solves the block triangle transposed.  x_p is written back into y.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_bwd(KArgs a, const int32_t* fronts, void* y, int nrhs,
                                                   const int* flag) {
  typedef typename Cx<R>::T C;
  if (done(flag)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* X = reinterpret_cast<C*>(smem_raw);
  const int s = blockIdx.y;
  const int f = fronts[blockIdx.x];
  const int p = a.npiv[f], u = a.nupd[f], m = p + u;
  C* T = X + (int64_t)m * nrhs;  // 64 x 65 transposed block triangle
  const int pb = a.pbeg[f];
  const C* L = (const C*)a.fac + (int64_t)s * a.fac_total + a.fac_off[f];
  C* Y = (C*)y + (int64_t)s * nrhs * a.N;
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
    const int k0 = ((k1 - 1) / 64) * 64;
    const int kn = k1 - k0;
    // X[k] -= sum_{i >= k1} L[i][k] X[i]   (one wave per column k, lanes over i)
    for (int k = k0 + wave; k < k1; k += NW) {
      for (int col = 0; col < nrhs; ++col) {
        C acc = czero<C>();
        for (int i = k1 + lane; i < m; i += 64)
          acc = cadd(acc, cmul(L[(int64_t)k * m + i], X[col * m + i]));
        for (int o = 32; o > 0; o >>= 1) {
          acc.x += __shfl_xor(acc.x, o);
          acc.y += __shfl_xor(acc.y, o);
        }
        if (lane == 0) X[col * m + k] = csub(X[col * m + k], acc);
      }
    }
    // stage the block triangle: T[l*65 + k] = L[k0+k][k0+l] (row k, column l)
    for (int idx = threadIdx.x; idx < kn * kn; idx += kThreads) {
      const int l = idx / kn, k = idx - l * kn;
      T[l * 65 + k] = L[(int64_t)(k0 + l) * m + k0 + k];
    }
    __syncthreads();
    if (wave == 0) {
      for (int col = 0; col < nrhs; ++col) {
        C v = lane < kn ? X[col * m + k0 + lane] : czero<C>();
        for (int k = kn - 1; k > 0; --k) {
          const C xk = shfl_c(v, k);
          if (lane < k) v = cfms(v, T[lane * 65 + k], xk);
        }
        if (lane < kn) X[col * m + k0 + lane] = v;
      }
    }
    __syncthreads();
    k1 = k0;
  }
  for (int idx = threadIdx.x; idx < p * nrhs; idx += kThreads) {
    const int col = idx / p, r = idx - col * p;
    Y[(int64_t)col * a.N + pb + r] = X[col * m + r];
  }
}

// ---------------------------------------------------------------------------
// FP64 refinement: r = rhs_sym - (SA) x, norms, convergence flag.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_residual(KArgs a, const double2* rhs, const double2* x,
                                                        double2* res, double* partial, int nrhs,
                                                        int scale_rhs, const int* flag) {
  if (done(flag)) return;
  const int col = blockIdx.y;
  const int s = col / nrhs;
  const double2* X = x + (int64_t)col * a.N;
  const double2* B = rhs + (int64_t)col * a.N;
  double2* Rv = res + (int64_t)col * a.N;
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
    if (scale_rhs) b = dmul(b, sym_scale(a, s, (int)n));
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
    double* pp = partial + ((int64_t)col * gridDim.x + blockIdx.x) * 2;
    pp[0] = red[0][0];
    pp[1] = red[1][0];
  }
}

__global__ void k_ir_begin(DevStatus* st) {
  st->ir_flag = 0;
  st->ir_steps = 0;
  st->ir_failed = 0;
  st->ir_rel = -1.0;
}

// One workgroup: per-column relative residuals in fixed order; sets the flag
// when every column meets tol (or a non-finite value stops the refinement).
__global__ __launch_bounds__(kThreads) void k_ir_check(DevStatus* st, const double* partial, int nblk,
                                                        int ncols, double tol, int step, int last) {
  if (st->ir_flag) return;
  __shared__ double worst[kThreads];
  __shared__ int bad[kThreads];
  double w = 0.0;
  int nf = 0;
  for (int col = threadIdx.x; col < ncols; col += kThreads) {
    double rr = 0.0, bb = 0.0;
    for (int b = 0; b < nblk; ++b) {
      rr += partial[((int64_t)col * nblk + b) * 2];
      bb += partial[((int64_t)col * nblk + b) * 2 + 1];
    }
    const double rel = bb > 0 ? sqrt(rr / bb) : sqrt(rr);
    if (!(rel <= DBL_MAX)) nf = 1;
    w = fmax(w, rel);
  }
  worst[threadIdx.x] = w;
  bad[threadIdx.x] = nf;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    int anybad = 0;
    for (int t = 0; t < kThreads; ++t) {
      mx = fmax(mx, worst[t]);
      anybad |= bad[t];
    }
    st->ir_rel = anybad ? NAN : mx;
    st->ir_steps = step;
    if (anybad) {
      st->nonfinite = 1;
      st->ir_failed = 1;
      st->ir_flag = 1;
    } else if (mx <= tol) {
      st->ir_flag = 1;
    } else if (last) {
      st->ir_failed = 1;
    }
  }
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
  return a;
}

inline unsigned grid1d(int64_t n, int64_t cap = 2048) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

template <typename R>
hipError_t refactor_impl(Plan& P, const double* eps, int64_t eps_stride, hipStream_t st) {
  const KArgs a = make_args(P);
  const int nsys = P.desc.nsys;
  const size_t cs = P.csize;
  const int NB = P.nb_large;
  Omegas om;
  for (int s = 0; s < kMaxSys; ++s) om.w[s] = s < nsys ? P.omega_host[s] : 0.0;
  hipLaunchKernelGGL(k_copy_eps, dim3(grid1d(P.an.N, 1024), nsys), dim3(kThreads), 0, st, a, eps,
                     eps_stride);
  hipLaunchKernelGGL(k_setup, dim3(nsys), dim3(kThreads), 0, st, a, om, P.desc.npml_x,
                     P.desc.npml_y);
  hipLaunchKernelGGL(k_anorm, dim3(grid1d(P.an.N, 512), nsys), dim3(kThreads), 0, st, a);
  const int32_t* lf = P.t.level_fronts;
  const int32_t* tk = P.t.tasks;
  for (const LevelPlan& L : P.levels) {
    if (L.small) {
      hipLaunchKernelGGL(k_front_small<R>, dim3(L.count, nsys), dim3(kThreads), L.small_lds, st, a,
                         lf + L.first);
      continue;
    }
    hipLaunchKernelGGL(k_assemble_large<R>, dim3(L.nasm, nsys), dim3(kThreads), 0, st, a,
                       tk + L.asm_off);
    for (const BlockStep& S : L.steps) {
      hipLaunchKernelGGL(k_diag_large<R>, dim3(S.ndiag, nsys), dim3(kThreads),
                         (size_t)(NB * NB + 2 * NB) * cs, st, a, tk + S.diag_off, S.kb);
      if (S.ntrsm)
        hipLaunchKernelGGL(k_trsm_large<R>, dim3(S.ntrsm, nsys), dim3(kThreads),
                           (size_t)(NB * NB + 64 * NB + NB) * cs, st, a, tk + S.trsm_off, S.kb);
      if (S.nupd)
        hipLaunchKernelGGL(k_update_large<R>, dim3(S.nupd, nsys), dim3(kThreads),
                           (size_t)(2 * NB * 64) * cs, st, a, tk + S.upd_off, S.kb);
    }
  }
  return hipGetLastError();
}

template <typename R>
void sweep(Plan& P, const KArgs& a, const double2* src, double2* dst, int nrhs, int scale_in,
           int accumulate, const int* flag, hipStream_t st) {
  const int nsys = P.desc.nsys;
  const int ncols = nsys * nrhs;
  const size_t cs = P.csize;
  hipLaunchKernelGGL(k_gather<R>, dim3(grid1d(P.an.N, 1024), ncols), dim3(kThreads), 0, st, a, src,
                     P.y, nrhs, scale_in, flag);
  const int32_t* lf = P.t.level_fronts;
  for (size_t l = 0; l < P.levels.size(); ++l) {
    const LevelPlan& L = P.levels[l];
    hipLaunchKernelGGL(k_fwd<R>, dim3(L.count, nsys), dim3(kThreads), (size_t)L.max_m * nrhs * cs, st,
                       a, lf + L.first, P.y, P.wv, nrhs, flag);
  }
  for (size_t l = P.levels.size(); l-- > 0;) {
    const LevelPlan& L = P.levels[l];
    hipLaunchKernelGGL(k_bwd<R>, dim3(L.count, nsys), dim3(kThreads),
                       ((size_t)L.max_m * nrhs + 64 * 65) * cs, st, a, lf + L.first, P.y, nrhs, flag);
  }
  hipLaunchKernelGGL(k_scatter<R>, dim3(grid1d(P.an.N, 1024), ncols), dim3(kThreads), 0, st, a, P.y,
                     dst, nrhs, accumulate, 0, flag);
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
  for (int it = 1; it <= max_ir; ++it) {
    hipLaunchKernelGGL(k_residual, dim3(P.res_blocks, ncols), dim3(kThreads), 0, st, a, rhs, xdst,
                       P.res, P.partial, nrhs, scale, flag);
    hipLaunchKernelGGL(k_ir_check, dim3(1), dim3(kThreads), 0, st, P.status, P.partial, P.res_blocks,
                       ncols, tol, it - 1, 0);
    sweep<R>(P, a, P.res, xdst, nrhs, 0, 1, flag, st);
  }
  if (max_ir > 0) {
    hipLaunchKernelGGL(k_residual, dim3(P.res_blocks, ncols), dim3(kThreads), 0, st, a, rhs, xdst,
                       P.res, P.partial, nrhs, scale, flag);
    hipLaunchKernelGGL(k_ir_check, dim3(1), dim3(kThreads), 0, st, P.status, P.partial, P.res_blocks,
                       ncols, tol, max_ir, 1);
  }
  hipLaunchKernelGGL(k_ir_end, dim3(1), dim3(1), 0, st, P.status, mode, max_ir > 0 ? 1 : 0);
  return hipGetLastError();
}

template <typename R>
hipError_t set_lds_limits(int limit) {
  hipError_t e = hipSuccess;
  const void* fns[] = {(const void*)k_front_small<R>, (const void*)k_diag_large<R>,
                       (const void*)k_trsm_large<R>, (const void*)k_update_large<R>,
                       (const void*)k_fwd<R>, (const void*)k_bwd<R>};
  for (const void* fn : fns) {
    hipError_t r = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, limit);
    if (r != hipSuccess && e == hipSuccess) e = r;
  }
  return e;
}

}  // namespace

hipError_t configure_kernels(Plan& P, int lds_limit) {
  return P.is_c64 ? set_lds_limits<float>(lds_limit) : set_lds_limits<double>(lds_limit);
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
