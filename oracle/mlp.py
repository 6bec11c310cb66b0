"""fp64 oracle of the learned-bucket form's CDF model -- TEST INFRASTRUCTURE ONLY.

The paper has no learned component; the model below is this project's
definition of the "small two-layer MLP CDF model" of the learned-bucket form.
The GPU trains the same model in FP32 with hand-written kernels; this module
is the plain fp64 statement of the same arithmetic that those kernels are
checked against (gradients, one Adam step, the trained loss).

Model (H hidden units, H even; parameter vector theta of length 3H+1 laid
out as [p_0..p_{H-1}, b1_0..b1_{H-1}, q_0..q_{H-1}, b2]):

    s_h  = +1 for h < H/2, -1 otherwise       (fixed signs)
    w1_h = s_h * softplus(p_h),  w2_h = s_h * softplus(q_h)
    F(x) = b2 + sum_h w2_h * relu(w1_h * x + b1_h)

Every unit has w1_h * w2_h >= 0, so F is non-decreasing in x: the model is
monotone by construction, and so are the bucket ids derived from it.

Loss over a sorted sample x_0 <= ... <= x_{S-1} with targets
y_i = (i + 0.5) / S (the mid-rank of each sample position):

    L = (1/S) * sum_i (F(x_i) - y_i)^2

Optimiser: Adam (beta1 = 0.9, beta2 = 0.999, eps = 1e-8) with bias
correction, a fixed step count and a fixed learning rate.

Input features are computed from the integer key in float32, exactly as the
GPU computes them (IEEE round-to-nearest-even), so both sides see
bit-identical x:
    linear:  x = fl32(k) * 2^-32
    log:     x = (bits(fl32(fl32(k) + 1)) - bits(1.0f)) * 2^-28   (a monotone
             piecewise-linear approximation of log2(1 + k) / 32)
"""
import numpy as np

BETA1 = 0.9
BETA2 = 0.999
EPS = 1e-8


def signs(H: int) -> np.ndarray:
    s = np.ones(H)
    s[H // 2:] = -1.0
    return s


def softplus(v):
    return np.logaddexp(0.0, v)


def sigmoid(v):
    return 0.5 * (1.0 + np.tanh(0.5 * v))


def unpack(theta: np.ndarray, H: int):
    theta = np.asarray(theta, np.float64)
    assert theta.size == 3 * H + 1
    return theta[:H], theta[H:2 * H], theta[2 * H:3 * H], theta[3 * H]


def weights(theta: np.ndarray, H: int):
    """(w1, b1, w2, b2) of the monotone parametrisation."""
    p, b1, q, b2 = unpack(theta, H)
    s = signs(H)
    return s * softplus(p), b1, s * softplus(q), b2


def forward(theta: np.ndarray, x: np.ndarray, H: int) -> np.ndarray:
    w1, b1, w2, b2 = weights(theta, H)
    z = np.outer(np.asarray(x, np.float64), w1) + b1
    return b2 + np.maximum(z, 0.0) @ w2


def targets(S: int) -> np.ndarray:
    return (np.arange(S, dtype=np.float64) + 0.5) / S


def loss(theta: np.ndarray, x: np.ndarray, y: np.ndarray, H: int) -> float:
    r = forward(theta, x, H) - y
    return float(np.mean(r * r))


def grad(theta: np.ndarray, x: np.ndarray, y: np.ndarray, H: int) -> np.ndarray:
    """Analytic gradient of the mean squared error w.r.t. theta (chain rule)."""
    x = np.asarray(x, np.float64)
    S = x.size
    p, b1, q, b2 = unpack(theta, H)
    s = signs(H)
    w1, w2 = s * softplus(p), s * softplus(q)
    z = np.outer(x, w1) + b1                 # (S, H)
    a = np.maximum(z, 0.0)
    r = (b2 + a @ w2 - y) * (2.0 / S)        # dL/dF per sample
    g_w2 = a.T @ r                           # dL/dw2_h
    g_z = np.outer(r, w2) * (z > 0.0)        # dL/dz_h (relu' = 1 where z > 0)
    g_b1 = g_z.sum(axis=0)
    g_w1 = g_z.T @ x
    g = np.empty(3 * H + 1)
    g[:H] = g_w1 * s * sigmoid(p)            # d softplus(p)/dp = sigmoid(p)
    g[H:2 * H] = g_b1
    g[2 * H:3 * H] = g_w2 * s * sigmoid(q)
    g[3 * H] = r.sum()
    return g


def adam_step(theta, g, m, v, t: int, lr: float):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * g
    v = BETA2 * v + (1.0 - BETA2) * g * g
    mh = m / (1.0 - BETA1 ** t)
    vh = v / (1.0 - BETA2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + EPS), m, v


def init_params(x_sorted: np.ndarray, H: int, slope: float = 1.0, out_w: float = 0.1) -> np.ndarray:
    """Deterministic start point from the sorted sample.

    Unit h gets |w1| = slope and its ReLU kink at the sample quantile
    (h + 0.5) / H of x (rising units, s = +1, are active right of the kink,
    falling units, s = -1, left of it); |w2| = out_w; b2 = 0.5.
    """
    x = np.asarray(x_sorted, np.float64)
    S = x.size
    s = signs(H)
    knots = x[np.minimum(((np.arange(H) + 0.5) / H * S).astype(np.int64), S - 1)]
    p = np.full(H, np.log(np.expm1(slope)))
    q = np.full(H, np.log(np.expm1(out_w)))
    b1 = -s * slope * knots
    return np.concatenate([p, b1, q, [0.5]])


def train(x_sorted: np.ndarray, H: int, steps: int, lr: float, theta0=None):
    """Full-batch Adam on the sorted sample; returns (theta, loss history)."""
    x = np.asarray(x_sorted, np.float64)
    y = targets(x.size)
    theta = init_params(x, H) if theta0 is None else np.array(theta0, np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    hist = []
    for t in range(1, steps + 1):
        g = grad(theta, x, y, H)
        hist.append(loss(theta, x, y, H))
        theta, m, v = adam_step(theta, g, m, v, t, lr)
    hist.append(loss(theta, x, y, H))
    return theta, np.array(hist)


def feature_linear(keys: np.ndarray) -> np.ndarray:
    k = np.asarray(keys, np.uint32)
    return (k.astype(np.float32) * np.float32(2.0 ** -32)).astype(np.float32)


def feature_log(keys: np.ndarray) -> np.ndarray:
    k = np.asarray(keys, np.uint32)
    f = k.astype(np.float32) + np.float32(1.0)
    bits = f.view(np.uint32).astype(np.int64) - 0x3F800000
    return (bits.astype(np.int32).astype(np.float32) * np.float32(2.0 ** -28)).astype(np.float32)


def bucket_ids(theta: np.ndarray, x: np.ndarray, H: int, B: int) -> np.ndarray:
    """b = clamp(floor(F(x) * B), 0, B - 1), evaluated in fp64 (speed-only role)."""
    u = forward(theta, x, H) * B
    return np.clip(np.floor(u), 0, B - 1).astype(np.int64)
