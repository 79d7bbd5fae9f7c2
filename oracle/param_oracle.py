"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Plain reference of the design parametrisation that maps the optimiser's
variables theta (one per design pixel, in [0, 1]) to the permittivity of the
design block (paper Sec. III and Sec. IV: a smoothing filter of 200 nm radius
followed by a sigmoid-like projection that pushes the design towards two
materials).  Only the tests may call it; the GPU library never does and shares
no code with it.

Readings (the paper names the two operations and the radius only):
  * filter: conic (linear hat) weights w(d) = max(0, 1 - d/R) of the distance d
    between pixel centres (cells), R = radius / dx, taken over the pixels of
    the design block only and normalised per output pixel by the sum of the
    weights it used:  rho~_i = sum_j w(d_ij) theta_j / sum_j w(d_ij);
  * projection: the tanh threshold projection with steepness beta and
    threshold eta:  P(x) = (tanh(beta eta) + tanh(beta (x - eta)))
                         / (tanh(beta eta) + tanh(beta (1 - eta)));
  * material: eps = eps_min + P(rho~) (eps_max - eps_min).
The backward pass is the chain rule through those three maps; the filter's
transpose is  (W^T y)_j = sum_i w(d_ij) y_i / S_i  with S_i = sum_k w(d_ik).
"""
from __future__ import annotations

import numpy as np


def _offsets(radius):
    """(di, dj, w) of every tap with w(d) > 0 for a radius in cells."""
    r = int(np.ceil(radius))
    taps = []
    for dj in range(-r, r + 1):
        for di in range(-r, r + 1):
            w = 1.0 - np.hypot(di, dj) / radius
            if w > 0.0:
                taps.append((di, dj, w))
    return taps


def _shifted_sum(field, radius):
    """sum_j w(d_ij) field_j over the block, field of shape (h, w), by taps."""
    h, w_ = field.shape
    out = np.zeros_like(field, dtype=np.float64)
    for di, dj, w in _offsets(radius):
        # out[j, i] += w * field[j + dj, i + di] where both inside the block
        j0, j1 = max(0, -dj), min(h, h - dj)
        i0, i1 = max(0, -di), min(w_, w_ - di)
        if j0 < j1 and i0 < i1:
            out[j0:j1, i0:i1] += w * field[j0 + dj:j1 + dj, i0 + di:i1 + di]
    return out


def weight_sums(shape, radius):
    """S_i = sum of the conic weights each pixel of the block uses."""
    return _shifted_sum(np.ones(shape), radius)


def conic_filter(theta, radius):
    """rho~ = W theta with per-pixel normalisation (theta: (h, w))."""
    theta = np.asarray(theta, dtype=np.float64)
    return _shifted_sum(theta, radius) / weight_sums(theta.shape, radius)


def conic_filter_transpose(y, radius):
    """W^T y: the conic weights are symmetric in the pixel pair, so this is
    the same weighted sum applied to y / S."""
    y = np.asarray(y, dtype=np.float64)
    return _shifted_sum(y / weight_sums(y.shape, radius), radius)


def tanh_projection(x, beta, eta):
    num = np.tanh(beta * eta) + np.tanh(beta * (np.asarray(x, dtype=np.float64) - eta))
    return num / (np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta)))


def tanh_projection_derivative(x, beta, eta):
    """dP/dx = beta sech^2(beta (x - eta)) / (tanh(beta eta) + tanh(beta (1 - eta)))."""
    c = np.cosh(beta * (np.asarray(x, dtype=np.float64) - eta))
    return beta / (c * c) / (np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta)))


def design_eps(theta, radius, beta, eta, eps_min, eps_max):
    """theta (h, w) -> (rho~, eps of the design block)."""
    rho = conic_filter(theta, radius)
    return rho, eps_min + tanh_projection(rho, beta, eta) * (eps_max - eps_min)


def design_eps_backward(rho, grad_eps, radius, beta, eta, eps_min, eps_max):
    """dF/dtheta from dF/deps on the design block (chain rule, reverse order)."""
    g = np.asarray(grad_eps, dtype=np.float64) * (eps_max - eps_min)
    g = g * tanh_projection_derivative(rho, beta, eta)
    return conic_filter_transpose(g, radius)
