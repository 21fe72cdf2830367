"""Pins of the learned-initial-guess reference (oracle.guess): grid transfers by
exact reproduction properties, the perceptron by a hand-built network with a
closed-form output, its gradients by central differences and by the optimality
of a least-squares fit, Adam by its bias-corrected constant-gradient step."""
import numpy as np
import pytest

from oracle import guess as G


@pytest.mark.parametrize("n,nc", [(16, 4), (256, 32), (24, 3)])
def test_restriction_of_constants_and_linear_functions(n, nc):
    h = 1.0 / (n + 1)
    r = n // nc
    t = (np.arange(n) + 1) * h
    X, Y = np.meshgrid(t, t, indexing="xy")
    assert np.allclose(G.restrict(np.full(n * n, 3.5), n, nc), 3.5, rtol=0, atol=1e-15)
    # mean of (i+1) h over block I is (I r + (r+1)/2) h
    want = (np.arange(nc) * r + (r + 1) / 2.0) * h
    got = G.restrict(X.ravel(), n, nc).reshape(nc, nc)
    assert np.allclose(got, want[None, :], rtol=0, atol=1e-15)
    got = G.restrict(Y.ravel(), n, nc).reshape(nc, nc)
    assert np.allclose(got, want[:, None], rtol=0, atol=1e-15)


@pytest.mark.parametrize("n,nc", [(16, 4), (256, 32)])
def test_prolongation_reproduces_linear_functions_between_centres(n, nc):
    h = 1.0 / (n + 1)
    r = n // nc
    t = (np.arange(n) + 1) * h
    c = (np.arange(nc) * r + (r - 1) / 2.0 + 1.0) * h       # centre of block I
    inside = (t >= c[0]) & (t <= c[-1])
    for fc, ff in [(np.ones((nc, nc)), lambda X, Y: np.ones_like(X)),
                   (np.tile(c, (nc, 1)), lambda X, Y: X),
                   (np.tile(c[:, None], (1, nc)), lambda X, Y: Y),
                   (2.0 + c[None, :] - 3.0 * c[:, None], lambda X, Y: 2.0 + X - 3.0 * Y)]:
        fine = G.prolong(fc.ravel(), n, nc).reshape(n, n)
        X, Y = np.meshgrid(t, t, indexing="xy")
        m = inside[None, :] & inside[:, None]
        assert np.allclose(fine[m], ff(X, Y)[m], rtol=0, atol=1e-13)
    # outside the band the interpolant falls linearly to zero at the boundary
    ones = G.prolong(np.ones(nc * nc), n, nc).reshape(n, n)
    left = t < c[0]
    assert np.allclose(ones[n // 2, left], t[left] / c[0], rtol=0, atol=1e-14)
    right = t > c[-1]
    assert np.allclose(ones[n // 2, right], (1.0 - t[right]) / (1.0 - c[-1]), rtol=0, atol=1e-14)


def test_prolongation_of_a_coarse_delta_is_a_product_of_tents():
    n, nc = 32, 4
    h = 1.0 / (n + 1)
    r = n // nc
    t = (np.arange(n) + 1) * h
    nodes = np.concatenate([[0.0], (np.arange(nc) * r + (r - 1) / 2.0 + 1.0) * h, [1.0]])
    for I, J in [(0, 0), (1, 2), (3, 3)]:
        d = np.zeros((nc, nc))
        d[J, I] = 1.0                                         # row = y index
        fine = G.prolong(d.ravel(), n, nc).reshape(n, n)
        tent = lambda x, k: np.clip(np.minimum((x - nodes[k]) / (nodes[k + 1] - nodes[k]),
                                               (nodes[k + 2] - x) / (nodes[k + 2] - nodes[k + 1])),
                                    0.0, None)
        want = tent(t, J)[:, None] * tent(t, I)[None, :]
        assert np.allclose(fine, want, rtol=0, atol=1e-14)


def test_features_are_scale_invariant():
    rng = np.random.default_rng(0)
    n, nc, fdim = 64, 8, 80
    b = rng.standard_normal(n * n)
    p = rng.standard_normal(10)
    f1, s1 = G.features(b, p, n, nc, fdim)
    f2, s2 = G.features(7.5 * b, p, n, nc, fdim)
    assert np.allclose(f1, f2, rtol=1e-14, atol=1e-15) and np.isclose(s2, 7.5 * s1, rtol=1e-14)
    assert np.isclose(np.mean(f1[:nc * nc] ** 2), 1.0, rtol=1e-14)
    assert np.array_equal(f1[nc * nc:nc * nc + 10], p) and not f1[nc * nc + 10:].any()
    f0, s0 = G.features(np.zeros(n * n), p, n, nc, fdim)
    assert s0 == 0.0 and not f0[:nc * nc].any()


def test_forward_of_a_hand_built_absolute_value_network():
    # |x| = relu(x) + relu(-x); a second input channel is ignored
    W1 = np.array([[1.0, -1.0], [0.0, 0.0]])
    W2 = np.array([[1.0], [1.0]])
    params = [(W1, np.zeros(2)), (W2, np.array([0.25]))]
    X = np.array([[-3.0, 9.0], [0.0, 1.0], [2.5, -4.0]])
    _, Y = G.forward(params, X)
    assert np.array_equal(Y[:, 0], np.abs(X[:, 0]) + 0.25)


def _rand_params(widths, rng):
    return [(rng.standard_normal((a, b)) * np.sqrt(2.0 / a), 0.1 * rng.standard_normal(b))
            for a, b in zip(widths[:-1], widths[1:])]


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    widths = [5, 7, 6, 3]
    params = _rand_params(widths, rng)
    X = rng.standard_normal((4, 5))
    T = rng.standard_normal((4, 3))
    _, grads = G.gradients(params, X, T)
    eps = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            for idx in np.ndindex(arr.shape):
                old = arr[idx]
                arr[idx] = old + eps
                lp = G.mse(G.forward(params, X)[1], T)
                arr[idx] = old - eps
                lm = G.mse(G.forward(params, X)[1], T)
                arr[idx] = old
                assert abs((lp - lm) / (2 * eps) - g[idx]) <= 1e-7 * (1 + abs(g[idx])), (l, idx)


def test_gradient_vanishes_at_the_least_squares_fit():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((40, 6))
    T = rng.standard_normal((40, 3))
    coef, *_ = np.linalg.lstsq(np.hstack([X, np.ones((40, 1))]), T, rcond=None)
    params = [(coef[:6].copy(), coef[6].copy())]
    loss, grads = G.gradients(params, X, T)
    assert np.max(np.abs(grads[0][0])) <= 1e-14 and np.max(np.abs(grads[0][1])) <= 1e-14
    _, g_off = G.gradients([(coef[:6] + 0.01, coef[6].copy())], X, T)
    assert np.max(np.abs(g_off[0][0])) > 1e-4


def test_adam_constant_gradient_steps():
    # with a constant gradient the bias-corrected moments are exactly g and g^2,
    # so every step moves each entry by lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3])
    opt = G.Adam([g.shape], lr=0.01, eps=1e-8)
    theta = [np.zeros(3)]
    for t in range(1, 6):
        theta = opt.step(theta, [g])
        assert np.allclose(theta[0], -t * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
