"""Pins of the fp64 MLP CDF oracle: central finite differences, the
least-squares line (closed form) when every ReLU stays active, Adam's first
step in closed form, the start point interpolating the quantile knots, and
the inference table (exact where the network is monotone, monotone always).
CPU only."""
import numpy as np
import pytest

from oracle import mlp


def _rand_theta(rng, H):
    return rng.normal(size=3 * H + 1)


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
    th = np.concatenate([np.full(H, 1.0), np.full(H, 1.0), np.full(H, 0.3), [0.0]])
    th, hist = mlp.train(x, H, steps=4000, lr=1e-2, theta0=th)
    w1, b1, w2, b2 = mlp.unpack(th, H)
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


@pytest.mark.parametrize("H", [1, 4, 16])
def test_start_point_interpolates_the_quantile_knots(H):
    rng = np.random.default_rng(9)
    S = 4096
    x = np.sort(rng.gamma(2.0, 0.1, size=S))
    th = mlp.init_params(x, H)
    q = (np.arange(H + 1) * (S - 1)) // H
    np.testing.assert_allclose(mlp.forward(th, x[q], H), (q + 0.5) / S, rtol=0, atol=1e-12)
    # constant left of the first knot, linear between knots
    assert mlp.forward(th, [x[0] - 1.0], H)[0] == pytest.approx((0.5) / S)
    mid = 0.5 * (x[q[0]] + x[q[1]])
    lin = (0.5 + (q[1] + 0.5 - 0.5) * (mid - x[q[0]]) / (x[q[1]] - x[q[0]])) / S
    assert mlp.forward(th, [mid], H)[0] == pytest.approx(lin, rel=1e-12)


def test_start_point_with_ties_reaches_post_tie_values():
    x = np.sort(np.concatenate([np.full(600, 0.25), np.linspace(0.3, 0.9, 424)]))
    H = 8
    th = mlp.init_params(x, H)
    k, yk = mlp.quantile_knots(x, H)
    last_of_run = np.r_[k[:-1] < k[1:], True]
    np.testing.assert_allclose(mlp.forward(th, k[last_of_run], H), yk[last_of_run], atol=1e-12)


def test_pl_table_exact_for_monotone_networks_and_monotone_always():
    rng = np.random.default_rng(10)
    S = 1000
    lo, hi = 0.5 / S, 1 - 0.5 / S
    for _ in range(40):
        H = int(rng.choice([2, 4, 16]))
        x_min, x_max = sorted(rng.uniform(0, 1, 2))
        xs = np.linspace(x_min, x_max, 20001)
        # a non-decreasing network that stays inside (lo, hi) on the range
        th = np.concatenate([rng.uniform(0.1, 3, H), rng.uniform(-2, 1, H), rng.uniform(0.01, 1, H), [0.0]])
        F = mlp.forward(th, xs, H)                       # b2 = 0 here
        th[2 * H:3 * H] *= 0.4 / max(F[-1] - F[0], 1e-12)
        th[3 * H] = 0.3 - mlp.forward(th, xs[:1], H)[0]   # F spans [0.3, 0.7] on the range
        F = mlp.forward(th, xs, H)
        tab = mlp.pl_table(th, H, x_min, x_max, S)
        ev = mlp.pl_eval(tab, xs)
        inner = slice(1, -1)   # the ends are pinned to lo / hi
        np.testing.assert_allclose(ev[inner][(xs[inner] > tab[0][1]) & (xs[inner] < tab[0][-2])],
                                   F[inner][(xs[inner] > tab[0][1]) & (xs[inner] < tab[0][-2])],
                                   rtol=1e-12, atol=1e-12)
        assert tab[1][0] == lo and tab[1][-1] == hi
        # arbitrary network: non-decreasing, inside [lo, hi] on the range and
        # inside [0, 1] beyond it, running max at interior points
        th2 = rng.normal(scale=2.0, size=3 * H + 1)
        t, V = mlp.pl_table(th2, H, x_min, x_max, S)
        wide = np.linspace(-0.5, 1.5, 40001)
        ev = mlp.pl_eval((t, V), wide)
        assert (np.diff(ev) >= 0).all() and ev.min() >= 0 and ev.max() <= 1
        inside = (wide >= x_min) & (wide <= x_max)
        assert ev[inside].min() >= lo and ev[inside].max() <= hi
        dense = np.linspace(x_min, x_max, 200001)
        runmax = np.clip(np.maximum.accumulate(mlp.forward(th2, dense, H)), lo, hi)
        np.testing.assert_allclose(V[1:-1], np.interp(t[1:-1], dense, runmax), atol=1e-3 * (1 + np.abs(V).max()))


def test_pl_table_ends_spread_the_tails():
    """A network that overshoots 1 before the sample maximum would send the
    whole upper tail to the last bucket; the pinned ends spread it."""
    H = 2
    th = np.array([1.0, 0.0, 0.0, 0.0, 2.0, 0.0, 0.0])   # F(x) = 2x
    x_min, x_max, S = 0.0, 1.0, 1 << 16
    xs = np.linspace(0.5, 1.0, 1001)                     # F >= 1 on all of these
    b = mlp.bucket_ids(mlp.pl_table(th, H, x_min, x_max, S), xs, 1024)
    assert np.unique(b).size > 500


def test_pl_table_has_no_flat_segment():
    """A network that reaches the upper clamp at an interior breakpoint, or
    is flat between two, would leave a flat segment holding every key of its
    x range in one bucket; those points are dropped and every segment of the
    table rises."""
    H = 3
    # F(x) = 4 relu(x - 0.1) - 4 relu(x - 0.3) + 2 relu(x - 0.6): rises on
    # [0.1, 0.3], flat on [0.3, 0.6], rises past 1 by x = 0.9
    th = np.array([1.0, 1.0, 1.0, -0.1, -0.3, -0.6, 4.0, -4.0, 2.0, 0.0])
    S = 1 << 10
    t, V = mlp.pl_table(th, H, 0.0, 1.0, S)
    assert t[0] == 0.0 and t[-1] == 1.0
    assert (np.diff(V) > 0).all(), (t, V)
    assert 0.6 not in t.tolist()     # flat after 0.3: dropped
    # keys spread over [0.3, 1.0] instead of piling up at one value
    xs = np.linspace(0.31, 0.99, 1000)
    assert np.unique(mlp.bucket_ids((t, V), xs, 1 << 12)).size > 500


def test_pl_eval_continues_the_end_segments():
    """Beyond the sample's extremes the first and last segments continue
    with their slopes, clipped to [0, 1]: for uniform keys (F(x) = x on
    [0.25, 0.75]) a key above the range lands where the line puts it, and
    the keys beyond the ends spread over as many buckets as keys inside
    would, instead of piling into the end buckets."""
    S = 1000
    t = np.array([0.25, 0.5, 0.75])
    V = np.array([0.5 / S, 0.5, 1 - 0.5 / S])
    s_hi = (V[2] - V[1]) / 0.25
    s_lo = (V[1] - V[0]) / 0.25
    xs = np.array([0.0, 0.2499, 0.7501, 0.76, 2.0])
    got = mlp.pl_eval((t, V), xs)
    want = [max(0.0, V[0] - s_lo * 0.25), V[0] - s_lo * 0.0001, V[2] + s_hi * 0.0001,
            min(1.0, V[2] + s_hi * 0.01), 1.0]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)
    # 64 keys evenly past the top end, 0.5 / S of rank: with B = 64 S buckets
    # they fill B / (2 S) = 32 buckets, not one
    B = 64 * S
    top = 0.75 + (np.arange(64) + 0.5) / 64 * (0.5 / S) / s_hi
    assert np.unique(mlp.bucket_ids((t, V), top, B)).size == 32


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


def test_training_improves_on_the_start_point():
    rng = np.random.default_rng(11)
    S = 4096
    x = np.sort(np.concatenate([rng.normal(0.2, 0.03, S // 3), rng.normal(0.55, 0.1, S // 3),
                                rng.normal(0.8, 0.01, S - 2 * (S // 3))]).clip(0, 1))
    th0 = mlp.init_params(x, 16)
    l0 = mlp.loss(th0, x, mlp.targets(S), 16)
    th, hist = mlp.train(x, 16, steps=200, lr=1e-3)
    assert hist[0] == pytest.approx(l0)
    assert hist[-1] < l0
    b = mlp.bucket_ids(mlp.pl_table(th, 16, x[0], x[-1], S), x, 64)
    assert (np.diff(b) >= 0).all()
