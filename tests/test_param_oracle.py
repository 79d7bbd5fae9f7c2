"""Pins of the design-parametrisation oracle (smoothing filter + projection,
paper Sec. III / Sec. IV) against what the mathematics fixes, independent of
the oracle's own code paths:

  filter     partition of unity (a constant stays constant, edges included);
             mass conservation of an interior impulse; exact reproduction of a
             linear field away from the edges (a symmetric kernel has zero
             first moments); the eight symmetries of the square and the
             support of the impulse response; a hand-worked 1.5-cell case;
             the transpose against the dense matrix and the adjoint identity
  projection fixed end points, the symmetry of eta = 0.5, the linear limit
             beta -> 0, the step limit beta -> infinity, monotonicity, and the
             closed-form derivative against central differences
  chain      the backward pass against central differences of a scalar
             function of eps
Each planted mistake (on the CPU, in a copy of an oracle function) must fail a
pin.
"""
import numpy as np
import pytest

from oracle import param_oracle as po


def _rand(shape, seed):
    return np.random.default_rng([seed, 3]).uniform(0.0, 1.0, size=shape)


@pytest.mark.parametrize("radius", [1.5, 2.0, 5.0, 8.0])
def test_constant_field_is_unchanged(radius):
    for shape in ((30, 30), (17, 41), (5, 7)):
        out = po.conic_filter(np.full(shape, 0.37), radius)
        assert np.allclose(out, 0.37, atol=1e-15, rtol=0)


@pytest.mark.parametrize("radius", [1.5, 3.0, 5.0])
def test_interior_impulse_conserves_mass(radius):
    n = 41
    x = np.zeros((n, n))
    x[20, 20] = 1.0
    out = po.conic_filter(x, radius)
    assert abs(out.sum() - 1.0) < 1e-14
    # support: nothing at or beyond the radius
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    d = np.hypot(ii - 20, jj - 20)
    assert np.all(out[d >= radius] == 0.0)
    assert np.all(out[d < radius] > 0.0)


@pytest.mark.parametrize("radius", [2.0, 5.0])
def test_linear_field_is_reproduced_in_the_interior(radius):
    n = 40
    jj, ii = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    f = 0.3 * ii - 0.7 * jj + 2.0
    out = po.conic_filter(f, radius)
    r = int(np.ceil(radius))
    inner = (slice(2 * r, n - 2 * r), slice(2 * r, n - 2 * r))
    assert np.allclose(out[inner], f[inner], atol=1e-12, rtol=0)
    # near the edges the per-pixel normalisation cannot keep the slope
    assert not np.allclose(out[0, :], f[0, :], atol=1e-6)


def test_impulse_response_has_the_symmetries_of_the_square():
    n = 31
    x = np.zeros((n, n))
    x[15, 15] = 1.0
    out = po.conic_filter(x, 5.0)
    assert np.allclose(out, out[::-1, :], atol=1e-16)
    assert np.allclose(out, out[:, ::-1], atol=1e-16)
    assert np.allclose(out, out.T, atol=1e-16)
    # decreasing along an axis inside the support
    row = out[15, 15:21]
    assert np.all(np.diff(row) < 0)


def test_hand_worked_radius_one_and_a_half():
    """R = 1.5: taps at distance 0 (weight 1), 1 (weight 1/3) and sqrt(2)
    (weight 1 - sqrt(2)/1.5 = 0.05719095841793653); an interior pixel's weight
    sum is 1 + 4/3 + 4 * 0.05719095841793653 = 2.5621...; the corner pixel of
    a block sees only itself, one neighbour on each axis and one diagonal."""
    x = np.zeros((9, 9))
    x[4, 4] = 1.0
    out = po.conic_filter(x, 1.5)
    s = 1.0 + 4.0 / 3.0 + 4.0 * 0.05719095841793653
    assert abs(out[4, 4] - 1.0 / s) < 1e-15
    assert abs(out[4, 5] - (1.0 / 3.0) / s) < 1e-15
    assert abs(out[5, 5] - 0.05719095841793653 / s) < 1e-15
    s_corner = 1.0 + 2.0 / 3.0 + 0.05719095841793653
    assert abs(po.weight_sums((9, 9), 1.5)[0, 0] - s_corner) < 1e-15


@pytest.mark.parametrize("radius", [1.5, 3.0])
def test_transpose_is_the_dense_transpose(radius):
    h, w = 9, 11
    W = np.zeros((h * w, h * w))
    for k in range(h * w):
        e = np.zeros(h * w)
        e[k] = 1.0
        W[:, k] = po.conic_filter(e.reshape(h, w), radius).reshape(-1)
    y = _rand((h, w), 1)
    assert np.allclose(po.conic_filter_transpose(y, radius).reshape(-1), W.T @ y.reshape(-1), atol=1e-14)
    x = _rand((h, w), 2)
    lhs = np.vdot(po.conic_filter(x, radius), y)
    rhs = np.vdot(x, po.conic_filter_transpose(y, radius))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("beta,eta", [(1.0, 0.5), (8.0, 0.5), (32.0, 0.3), (64.0, 0.7)])
def test_projection_end_points_and_monotone(beta, eta):
    assert abs(po.tanh_projection(0.0, beta, eta)) < 1e-15
    assert abs(po.tanh_projection(1.0, beta, eta) - 1.0) < 1e-15
    x = np.linspace(0, 1, 1001)
    d = np.diff(po.tanh_projection(x, beta, eta))
    assert np.all(d >= 0)                                   # saturates to exact 0 / 1 at large beta
    assert np.all(d[np.abs(x[1:] - eta) < 0.1] > 0)


def test_projection_symmetry_and_limits():
    x = np.linspace(0, 1, 101)
    for beta in (2.0, 16.0):
        assert np.allclose(po.tanh_projection(1 - x, beta, 0.5), 1 - po.tanh_projection(x, beta, 0.5), atol=1e-15)
    assert np.allclose(po.tanh_projection(x, 1e-5, 0.4), x, atol=1e-9)
    step = po.tanh_projection(np.array([0.1, 0.39, 0.41, 0.9]), 2000.0, 0.4)
    assert np.allclose(step, [0, 0, 1, 1], atol=1e-8)


@pytest.mark.parametrize("beta,eta", [(1.0, 0.5), (8.0, 0.5), (32.0, 0.35)])
def test_projection_derivative(beta, eta):
    x = np.linspace(0.02, 0.98, 49)
    h = 1e-6
    fd = (po.tanh_projection(x + h, beta, eta) - po.tanh_projection(x - h, beta, eta)) / (2 * h)
    an = po.tanh_projection_derivative(x, beta, eta)
    assert np.allclose(an, fd, rtol=1e-6, atol=1e-8 * beta)


def test_chain_backward_matches_central_differences():
    h_, w_ = 14, 17
    theta = _rand((h_, w_), 5)
    c = np.random.default_rng([5, 4]).standard_normal((h_, w_))
    args = dict(radius=3.0, beta=6.0, eta=0.5, eps_min=2.085, eps_max=12.11)

    def F(th):
        _, eps = po.design_eps(th, **args)
        return float((c * eps * eps).sum())

    rho, eps = po.design_eps(theta, **args)
    g = po.design_eps_backward(rho, 2.0 * c * eps, **args)
    h = 1e-6
    rng = np.random.default_rng([5, 5])
    for _ in range(12):
        j, i = rng.integers(0, h_), rng.integers(0, w_)
        tp, tm = theta.copy(), theta.copy()
        tp[j, i] += h
        tm[j, i] -= h
        fd = (F(tp) - F(tm)) / (2 * h)
        assert abs(g[j, i] - fd) <= 1e-6 * max(1.0, abs(fd))


# -- planted mistakes ---------------------------------------------------------

def test_planted_unnormalised_filter_fails_partition_of_unity():
    bad = lambda th, r: po._shifted_sum(th, r) / po.weight_sums((41, 41), r)[20, 20]
    out = bad(np.full((30, 30), 0.37), 3.0)
    assert not np.allclose(out, 0.37, atol=1e-6)


def test_planted_off_centre_kernel_fails_linear_reproduction():
    def shifted(th, r):
        out = np.zeros_like(th)
        for di, dj, w in po._offsets(r):
            out += w * np.roll(np.roll(th, -(dj + 1), axis=0), -di, axis=1)
        return out / sum(w for _, _, w in po._offsets(r))
    n = 40
    jj, ii = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    f = 0.3 * ii - 0.7 * jj + 2.0
    inner = (slice(10, 30), slice(10, 30))
    assert not np.allclose(shifted(f, 3.0)[inner], f[inner], atol=1e-6)


def test_planted_transpose_without_normalisation_fails_adjoint_identity():
    x, y = _rand((9, 11), 2), _rand((9, 11), 1)
    lhs = np.vdot(po.conic_filter(x, 3.0), y)
    bad = po._shifted_sum(y, 3.0) / po.weight_sums(y.shape, 3.0)   # W applied instead of W^T
    assert abs(lhs - np.vdot(x, bad)) > 1e-6 * abs(lhs)


def test_planted_derivative_mistake_fails():
    x = np.linspace(0.02, 0.98, 49)
    h = 1e-6
    fd = (po.tanh_projection(x + h, 8.0, 0.5) - po.tanh_projection(x - h, 8.0, 0.5)) / (2 * h)
    c = np.cosh(8.0 * (x - 0.5))
    bad = 8.0 / c / (np.tanh(4.0) + np.tanh(4.0))   # sech instead of sech^2
    assert not np.allclose(bad, fd, rtol=1e-3)
