"""Pins of the fp64 MLP CDF oracle: central finite differences, the
least-squares line (closed form) when every ReLU stays active, Adam's first
step in closed form, monotonicity of the parametrisation, exact feature
values.  CPU only."""
import numpy as np
import pytest

from oracle import mlp


def _rand_theta(rng, H):
    th = rng.normal(size=3 * H + 1)
    th[H:2 * H] = rng.uniform(-0.5, 0.5, size=H)
    return th


@pytest.mark.parametrize("H", [2, 8, 16])
def test_gradient_matches_central_differences(H):
    rng = np.random.default_rng(H)
    S = 257
    x = np.sort(rng.uniform(0, 1, size=S))
    y = mlp.targets(S)
    th = _rand_theta(rng, H)
    g = mlp.grad(th, x, y, H)
    h = 1e-6
    fd = np.empty_like(th)
    for i in range(th.size):
        e = np.zeros_like(th); e[i] = h
        fd[i] = (mlp.loss(th + e, x, y, H) - mlp.loss(th - e, x, y, H)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8 * np.abs(g).max())


def test_all_units_active_converges_to_least_squares_line():
    """With every ReLU active on [0, 1], F(x) = slope * x + icpt; Adam on
    the MSE must reach the normal-equation solution of the line fit."""
    H = 4
    rng = np.random.default_rng(7)
    x = np.sort(rng.beta(2, 5, size=2000))
    y = mlp.targets(x.size)
    A = np.stack([x, np.ones_like(x)], 1)
    slope_ls, icpt_ls = np.linalg.solve(A.T @ A, A.T @ y)
    th = np.zeros(3 * H + 1)
    th[:H] = np.log(np.expm1(0.5))          # |w1| = 0.5
    th[H:2 * H] = 5.0                        # b1 = 5 > |w1| keeps z > 0 on [0, 1]
    th[2 * H:3 * H] = np.log(np.expm1(0.3))
    th[3 * H] = 0.0
    th, hist = mlp.train(x, H, steps=6000, lr=3e-3, theta0=th)
    w1, b1, w2, b2 = mlp.weights(th, H)
    assert (np.outer([0.0, 1.0], w1) + b1 > 0).all()
    slope = float(w2 @ w1)
    icpt = float(b2 + w2 @ b1)
    assert abs(slope - slope_ls) < 2e-3 * abs(slope_ls)
    assert abs(icpt - icpt_ls) < 2e-3
    resid = A @ np.array([slope_ls, icpt_ls]) - y
    assert hist[-1] == pytest.approx(np.mean(resid ** 2), rel=1e-3)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(8)
    th = rng.normal(size=9)
    g = rng.normal(size=9)
    th1, m, v = mlp.adam_step(th, g, np.zeros(9), np.zeros(9), 1, lr=0.01)
    # bias-corrected first moments are g and g^2, so the step is lr*g/(|g|+eps)
    np.testing.assert_allclose(th1, th - 0.01 * g / (np.abs(g) + mlp.EPS), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_model_is_monotone_for_any_parameters():
    rng = np.random.default_rng(9)
    xs = np.linspace(-0.5, 1.5, 4001)
    for _ in range(50):
        H = int(rng.choice([2, 4, 16]))
        th = rng.normal(scale=3.0, size=3 * H + 1)
        F = mlp.forward(th, xs, H)
        assert (np.diff(F) >= -1e-12).all()


def test_feature_values_and_monotonicity():
    k = np.array([0, 1, 3, 7, 255, 2 ** 24 - 1, 2 ** 31, 2 ** 32 - 1], np.uint32)
    lin = mlp.feature_linear(k)
    assert lin[0] == 0 and lin[6] == 0.5
    lg = mlp.feature_log(k)
    # exact at 2^j - 1: log2(2^j) / 32 = j / 32
    assert lg.tolist()[:6] == [0.0, 1 / 32, 2 / 32, 3 / 32, 8 / 32, 24 / 32]
    assert lg[-1] == 1.0
    rng = np.random.default_rng(10)
    r = np.sort(rng.integers(0, 2 ** 32, size=100_000, dtype=np.uint64).astype(np.uint32))
    assert (np.diff(mlp.feature_log(r)) >= 0).all() and (np.diff(mlp.feature_linear(r)) >= 0).all()
    # the log feature is within 0.0861/32 of log2(1 + k)/32 (piecewise-linear log2)
    err = mlp.feature_log(r).astype(np.float64) - np.log2(1.0 + r.astype(np.float64)) / 32
    assert np.abs(err).max() < 0.0861 / 32 + 1e-6


def test_training_fits_a_mixture_cdf():
    rng = np.random.default_rng(11)
    S = 4096
    comp = rng.integers(0, 3, size=S)
    x = np.sort(np.clip(rng.normal([0.2, 0.5, 0.7][0], 0.05, size=S) * (comp == 0)
                        + rng.normal(0.5, 0.1, size=S) * (comp == 1)
                        + rng.normal(0.8, 0.02, size=S) * (comp == 2), 0, 1))
    th, hist = mlp.train(x, 16, steps=400, lr=0.02)
    assert hist[-1] < hist[0] / 20
    b = mlp.bucket_ids(th, x, 16, 64)
    assert (np.diff(b) >= 0).all()
