// Design parametrisation on the GPU (paper Sec. III and Sec. IV): the map from
// the optimiser's variables theta (one per design pixel) to the permittivity
// of the design block, a smoothing filter of a given radius followed by a
// sigmoid-like projection onto the two materials, and its backward pass.
//   filter      rho~_i = sum_j w(d_ij) theta_j / S_i,  S_i = sum_j w(d_ij),
//               w(d) = max(0, 1 - d/R) over the pixels j of the block,
//               d the distance between pixel centres in cells;
//   projection  P(x) = (tanh(b e) + tanh(b (x - e))) / (tanh(b e) + tanh(b (1 - e)));
//   material    eps = eps_min + P(rho~) (eps_max - eps_min).
// Backward: dF/dtheta = W^T (P'(rho~) (eps_max - eps_min) dF/deps), and since
// w is symmetric in the pixel pair, (W^T y)_j = sum_i w(d_ij) (y_i / S_i):
// one pass forms y_i / S_i, a second the same conic sum as the forward filter.
//
// One kernel serves all three passes: a 16 x 16 tile of outputs per workgroup,
// the input tile with its halo of ceil(R) - 1 cells staged in LDS as (value,
// inside-the-block) pairs, the tap weights in an LDS table.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/fdfd.h"

namespace {

constexpr int kTile = 16;
constexpr int kMaxHalo = 11;  // radius up to 12 cells (300 nm at 25 nm)
constexpr int kSpan = kTile + 2 * kMaxHalo;

enum { kForward = 0, kBackScale = 1, kBackSum = 2 };

struct ParamArgs {
  int w, h, i0, j0, nx;
  int halo;           // ceil(R) - 1: largest tap offset with w > 0
  double inv_r;       // 1 / R
  double beta, eta, eps_min, eps_max, pnorm;  // pnorm = 1 / (tanh(b e) + tanh(b (1 - e)))
};

__device__ __forceinline__ double projection(const ParamArgs& p, double x) {
  return (tanh(p.beta * p.eta) + tanh(p.beta * (x - p.eta))) * p.pnorm;
}

__device__ __forceinline__ double projection_slope(const ParamArgs& p, double x) {
  const double c = cosh(p.beta * (x - p.eta));
  return p.beta / (c * c) * p.pnorm;
}

// mode kForward:   in = theta (block), out = rho (block), eps (grid) written
// mode kBackScale: in = dF/deps (grid, the block read), aux = rho (block),
//                  out = P'(rho) (eps_max - eps_min) dF/deps / S (block)
// mode kBackSum:   in = the kBackScale output (block), out = dF/dtheta (block)
template <int Mode>
__global__ __launch_bounds__(kTile * kTile) void k_conic(ParamArgs p, const double* in, const double* aux,
                                                        double* out, double* eps) {
  __shared__ double2 tile[kSpan * kSpan];
  __shared__ double wt[(2 * kMaxHalo + 1) * (2 * kMaxHalo + 1)];
  const int H = p.halo, span = kTile + 2 * H, nt = 2 * H + 1;
  const int bx = blockIdx.x * kTile, by = blockIdx.y * kTile;
  const int tid = threadIdx.x;
  for (int k = tid; k < nt * nt; k += kTile * kTile) {
    const int di = k % nt - H, dj = k / nt - H;
    wt[k] = fmax(0.0, 1.0 - sqrt((double)(di * di + dj * dj)) * p.inv_r);
  }
  // the input with its halo: (value, 1) inside the block, (0, 0) outside
  for (int k = tid; k < span * span; k += kTile * kTile) {
    const int li = k % span, lj = k / span;
    const int i = bx + li - H, j = by + lj - H;
    double2 v = make_double2(0.0, 0.0);
    if (i >= 0 && i < p.w && j >= 0 && j < p.h) {
      const double x = Mode == kBackScale ? in[(int64_t)(p.j0 + j) * p.nx + p.i0 + i] : in[(int64_t)j * p.w + i];
      v = make_double2(x, 1.0);
    }
    tile[k] = v;
  }
  __syncthreads();
  const int ti = tid % kTile, tj = tid / kTile;
  const int i = bx + ti, j = by + tj;
  if (i >= p.w || j >= p.h) return;
  double num = 0.0, den = 0.0;
  for (int dj = 0; dj < nt; ++dj) {
    const double2* row = tile + (tj + dj) * span + ti;
    const double* wr = wt + dj * nt;
    for (int di = 0; di < nt; ++di) {
      const double w = wr[di];
      const double2 v = row[di];
      num = fma(w, v.x, num);
      den = fma(w, v.y, den);
    }
  }
  const int64_t o = (int64_t)j * p.w + i;
  if (Mode == kForward) {
    const double rho = num / den;
    out[o] = rho;
    eps[(int64_t)(p.j0 + j) * p.nx + p.i0 + i] = p.eps_min + projection(p, rho) * (p.eps_max - p.eps_min);
  } else if (Mode == kBackScale) {
    // here num is unused: the centre value (dF/deps of this pixel) and S = den
    const double g = tile[(tj + H) * span + ti + H].x;
    out[o] = g * (p.eps_max - p.eps_min) * projection_slope(p, aux[o]) / den;
  } else {
    out[o] = num;
  }
}

const char* check(const fdfd_param_desc* d) {
  if (!d) return "desc is NULL";
  if (d->w < 1 || d->h < 1) return "the design block needs w, h >= 1";
  if (d->i0 < 0 || d->j0 < 0 || d->i0 + d->w > d->nx || d->j0 + d->h > d->ny)
    return "the design block must lie inside the nx x ny map";
  if (!(d->radius > 0.0) || d->radius > kMaxHalo + 1) return "radius must be in (0, 12] cells";
  if (!(d->beta > 0.0) || !std::isfinite(d->beta)) return "beta must be positive and finite";
  if (!(d->eta > 0.0 && d->eta < 1.0)) return "eta must be in (0, 1)";
  if (!std::isfinite(d->eps_min) || !std::isfinite(d->eps_max)) return "eps_min and eps_max must be finite";
  return nullptr;
}

ParamArgs make(const fdfd_param_desc* d) {
  ParamArgs p;
  p.w = d->w;
  p.h = d->h;
  p.i0 = d->i0;
  p.j0 = d->j0;
  p.nx = d->nx;
  p.halo = (int)std::ceil(d->radius) - 1;
  p.inv_r = 1.0 / d->radius;
  p.beta = d->beta;
  p.eta = d->eta;
  p.eps_min = d->eps_min;
  p.eps_max = d->eps_max;
  p.pnorm = 1.0 / (std::tanh(d->beta * d->eta) + std::tanh(d->beta * (1.0 - d->eta)));
  return p;
}

thread_local std::string g_param_error;

fdfd_status param_fail(const char* msg) {
  g_param_error = msg;
  return FDFD_ERR_ARG;
}

}  // namespace

extern "C" {

fdfd_status fdfd_param_forward(const fdfd_param_desc* d, const double* theta_dev, double* rho_dev, double* eps_dev,
                               void* hip_stream) {
  if (const char* e = check(d)) return param_fail(e);
  if (!theta_dev || !rho_dev || !eps_dev) return param_fail("theta_dev, rho_dev and eps_dev must be non-NULL");
  const ParamArgs p = make(d);
  const dim3 grid((p.w + kTile - 1) / kTile, (p.h + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_conic<kForward>, grid, dim3(kTile * kTile), 0, (hipStream_t)hip_stream, p, theta_dev,
                     (const double*)nullptr, rho_dev, eps_dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_param_error = hipGetErrorString(e);
    return FDFD_ERR_HIP;
  }
  return FDFD_OK;
}

fdfd_status fdfd_param_backward(const fdfd_param_desc* d, const double* rho_dev, const double* grad_eps_dev,
                                double* work_dev, double* grad_theta_dev, void* hip_stream) {
  if (const char* e = check(d)) return param_fail(e);
  if (!rho_dev || !grad_eps_dev || !work_dev || !grad_theta_dev)
    return param_fail("rho_dev, grad_eps_dev, work_dev and grad_theta_dev must be non-NULL");
  const ParamArgs p = make(d);
  const dim3 grid((p.w + kTile - 1) / kTile, (p.h + kTile - 1) / kTile);
  hipStream_t st = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_conic<kBackScale>, grid, dim3(kTile * kTile), 0, st, p, grad_eps_dev, rho_dev, work_dev,
                     (double*)nullptr);
  hipLaunchKernelGGL(k_conic<kBackSum>, grid, dim3(kTile * kTile), 0, st, p, (const double*)work_dev,
                     (const double*)nullptr, grad_theta_dev, (double*)nullptr);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_param_error = hipGetErrorString(e);
    return FDFD_ERR_HIP;
  }
  return FDFD_OK;
}

const char* fdfd_param_last_error(void) { return g_param_error.c_str(); }

}  // extern "C"
