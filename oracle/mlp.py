"""fp64 oracle of the learned-bucket form's CDF model -- TEST INFRASTRUCTURE ONLY.

The paper has no learned component; the model below is this project's
definition of the "small two-layer MLP CDF model" of the learned-bucket form.
The GPU trains the same model in FP32 with hand-written kernels; this module
is the plain fp64 statement of the same arithmetic that those kernels are
checked against (gradients, one Adam step, the trained loss, the inference
table).

Model (H hidden units; parameter vector theta of length 3H+1 laid out as
[w1_0..w1_{H-1}, b1_0..b1_{H-1}, w2_0..w2_{H-1}, b2]):

    F(x) = b2 + sum_h w2_h * relu(w1_h * x + b1_h)

Loss over a sorted sample x_0 <= ... <= x_{S-1} with targets
y_i = (i + 0.5) / S (the mid-rank of each sample position):

    L = (1/S) * sum_i (F(x_i) - y_i)^2

Optimiser: Adam (beta1 = 0.9, beta2 = 0.999, eps = 1e-8) with bias
correction, a fixed step count and a fixed learning rate.

Start point (closed form): the piecewise-linear interpolant of the sample's
empirical CDF through H knots at sample quantiles -- unit h is a ramp
relu(x - k_h) whose output weight is the slope change at knot k_h.

Inference: a 1-D two-layer ReLU network is a piecewise-linear function whose
breakpoints are -b1_h / w1_h.  `pl_table` restricts it to the sample's
feature range [x_min, x_max]: points x_min, the breakpoints strictly inside,
x_max; values the running maximum of F at those points (the smallest
non-decreasing function >= F there), clamped into [0.5/S, 1 - 0.5/S], with
the two ends pinned to 0.5/S and 1 - 0.5/S -- the mid-ranks of the sample's
own extremes; then every interior point whose value (as a float32, the
precision the table is stored in) is not above the previous kept point's, or
reaches the upper clamp, is dropped, so no segment is flat (a flat segment
would send all its keys to one bucket).  `pl_eval` finds x's segment (the first one for x below the
range, the last one above it) and interpolates linearly, capped at the next
point's value inside the range; beyond the ends the first and last segments
continue with their slopes, clipped to [0, 1].  Inside the range, wherever F
is non-decreasing and within the clamp, the table reproduces F; everywhere
it is non-decreasing, so bucket ids derived from it are ordered like the
keys.  (Pinning the ends keeps the thin tails of a distribution from
collapsing into the first and last bucket when the trained F over- or
undershoots there; continuing the end segments spreads the keys beyond the
sample's extremes -- about n / S of them at each end -- over the buckets of
the remaining rank 0.5 / S, where a clamp would put them all into one.)

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


def unpack(theta: np.ndarray, H: int):
    theta = np.asarray(theta, np.float64)
    assert theta.size == 3 * H + 1
    return theta[:H], theta[H:2 * H], theta[2 * H:3 * H], theta[3 * H]


def forward(theta: np.ndarray, x: np.ndarray, H: int) -> np.ndarray:
    w1, b1, w2, b2 = unpack(theta, H)
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
    w1, b1, w2, b2 = unpack(theta, H)
    z = np.outer(x, w1) + b1                 # (S, H)
    a = np.maximum(z, 0.0)
    r = (b2 + a @ w2 - y) * (2.0 / S)        # dL/dF per sample
    g_z = np.outer(r, w2) * (z > 0.0)        # dL/dz_h (relu' = 1 where z > 0)
    g = np.empty(3 * H + 1)
    g[:H] = g_z.T @ x                        # dL/dw1
    g[H:2 * H] = g_z.sum(axis=0)             # dL/db1
    g[2 * H:3 * H] = a.T @ r                 # dL/dw2
    g[3 * H] = r.sum()                       # dL/db2
    return g


def adam_step(theta, g, m, v, t: int, lr: float):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * g
    v = BETA2 * v + (1.0 - BETA2) * g * g
    mh = m / (1.0 - BETA1 ** t)
    vh = v / (1.0 - BETA2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + EPS), m, v


def quantile_knots(x_sorted: np.ndarray, H: int):
    """Knot i (i = 0..H) at sample position q_i = floor(i * (S - 1) / H) with
    value y_{q_i} = (q_i + 0.5) / S."""
    S = x_sorted.size
    q = (np.arange(H + 1) * (S - 1)) // H
    return np.asarray(x_sorted, np.float64)[q], (q + 0.5) / S


def init_params(x_sorted: np.ndarray, H: int) -> np.ndarray:
    """Closed-form start: F equals the piecewise-linear interpolant through the
    quantile knots on [k_0, k_last] (constant y_0 left of k_0).  Of a run of
    equal knots (ties in the sample) only the last is kept, so F reaches the
    value after the tie.  Unit h has w1 = 1, b1 = -k_h and w2 = the slope
    change at k_h; unused units have w2 = 0."""
    k, yk = quantile_knots(x_sorted, H)
    keep = np.ones(H + 1, bool)
    keep[:-1] = k[:-1] < k[1:]
    k, yk = k[keep], yk[keep]
    m = k.size - 1
    w1 = np.ones(H)
    b1 = np.full(H, -k[-1])
    w2 = np.zeros(H)
    if m >= 1:
        slopes = np.diff(yk) / np.diff(k)
        b1[:m] = -k[:m]
        w2[:m] = np.diff(np.concatenate([[0.0], slopes]))
    return np.concatenate([w1, b1, w2, [yk[0]]])


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


def pl_table(theta: np.ndarray, H: int, x_min: float, x_max: float, S: int):
    """(t, V) of the network on [x_min, x_max] as described in the header."""
    w1, b1, w2, b2 = unpack(theta, H)
    with np.errstate(divide="ignore", invalid="ignore"):
        bp = -b1 / w1
    bp = bp[(w1 != 0) & (bp > x_min) & (bp < x_max)]
    t = np.concatenate([[x_min], np.unique(bp), [x_max]])
    lo, hi = 0.5 / S, 1.0 - 0.5 / S
    V = np.clip(np.maximum.accumulate(forward(theta, t, H)), lo, hi)
    V[0], V[-1] = lo, hi
    keep = [0]   # compared as the float32 values the table stores
    f = V.astype(np.float32)
    for i in range(1, t.size - 1):
        if f[keep[-1]] < f[i] < np.float32(hi):
            keep.append(i)
    keep.append(t.size - 1)
    return t[keep], V[keep]


def pl_eval(table, x: np.ndarray) -> np.ndarray:
    """Monotone evaluation of a table: find x's segment (the first below
    t_0, the last above t_last), interpolate, cap at the segment's right
    value (1 for the last segment), floor at 0."""
    t, V = table
    x = np.asarray(x, np.float64)
    j = np.clip(np.searchsorted(t, x, side="right") - 1, 0, t.size - 2)
    dt = t[j + 1] - t[j]
    slope = np.where(dt > 0, (V[j + 1] - V[j]) / np.where(dt > 0, dt, 1.0), 0.0)
    cap = np.where(j == t.size - 2, 1.0, V[j + 1])
    return np.clip(V[j] + slope * (x - t[j]), 0.0, cap)


def feature_linear(keys: np.ndarray) -> np.ndarray:
    k = np.asarray(keys, np.uint32)
    return (k.astype(np.float32) * np.float32(2.0 ** -32)).astype(np.float32)


def feature_log(keys: np.ndarray) -> np.ndarray:
    k = np.asarray(keys, np.uint32)
    f = k.astype(np.float32) + np.float32(1.0)
    bits = f.view(np.uint32).astype(np.int64) - 0x3F800000
    return (bits.astype(np.int32).astype(np.float32) * np.float32(2.0 ** -28)).astype(np.float32)


def bucket_ids(table, x: np.ndarray, B: int) -> np.ndarray:
    """b = clamp(floor(pl_eval(x) * B), 0, B - 1), in fp64 (speed-only role)."""
    u = pl_eval(table, x) * B
    return np.clip(np.floor(u), 0, B - 1).astype(np.int64)
