"""Oracle (test infrastructure): FP64 reference of the guard-width surrogate network.

The paper states that a model giving the number of guard cells n_g as a
function of the solver order p, the time step and the cell size is crucial to
pick n_g (Sec. 1.4, with Sec. 2.2 on how n_g drives memory and cost); it gives
no such model.  The surrogate here is a small multilayer perceptron that maps
six features of a local-with-guards run to log10 of its truncation error
against the global solve:

    h1 = silu(W1 x + b1)      W1: 64 x 6
    h2 = silu(W2 h1 + b2)     W2: 64 x 64
    y  = W3 h2 + b3           W3: 1 x 64
    silu(z) = z / (1 + exp(-z))

trained on the mean squared error L = mean_s (y_s - t_s)^2 with Adam (Kingma &
Ba, 2015: first and second moment averages with bias correction).  The GPU
stores the weights in bfloat16 with FP32 master copies; this module takes
whatever weight values it is given (the tests pass the bfloat16-rounded ones)
and computes in FP64.

Parameter vector layout (shared by both sides as a documented format, not as
code): W1 (row-major, out x in), b1, W2, b2, W3, b3 -- 4673 values.
"""

from __future__ import annotations

import numpy as np

NIN, NH = 6, 64
SHAPES = (("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (1, NH)), ("b3", (1,)))
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Split a flat parameter vector into named arrays (views)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (NPARAM,)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(params) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    """d silu / dz = s(z) (1 + z (1 - s(z))), s the logistic function."""
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X):
    """Network output y (n,) and the intermediate values, for inputs X (n, 6)."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(z2)
    y = (h2 @ p["W3"].T)[:, 0] + p["b3"][0]
    return y, {"X": X, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def loss(theta, X, t):
    y, _ = forward(theta, X)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def loss_and_grad(theta, X, t):
    """MSE loss and its gradient with respect to the flat parameter vector (chain rule, layer by layer)."""
    p = unpack(theta)
    y, c = forward(theta, X)
    n = y.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / n  # dL/dy_s
    g = {}
    g["W3"] = dy[None, :] @ c["h2"]
    g["b3"] = np.array([dy.sum()])
    dz2 = (dy[:, None] * p["W3"][0][None, :]) * silu_grad(c["z2"])
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * silu_grad(c["z1"])
    g["W1"] = dz1.T @ c["X"]
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean((y - t) ** 2)), pack(g)


def adam(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1**t)
    vhat = v / (1.0 - beta2**t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits of
    an IEEE binary32 value; the 16 dropped bits are rounded to nearest with ties
    to even.  NaN is kept a quiet NaN.
    """
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    r = np.where(nan, (u | 0x00400000) & 0xFFFF0000, r)
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).reshape(a.shape)


# ---------------------------------------------------------------- labels and features
FLOOR = -16.0


def truncation_error(local_fields, global_fields):
    """log10 of max |local - global| / max |global| over all cells and E, B components, floored at -16.

    Both inputs are (6, nz, ny, nx) arrays of E and B on the global grid after
    the same number of steps; every global cell is the interior of exactly one
    sub-domain, so the maximum runs over all cells.
    """
    a = np.asarray(local_fields, dtype=np.float64)
    b = np.asarray(global_fields, dtype=np.float64)
    ref = np.abs(b).max()
    err = np.abs(a - b).max() / ref if ref > 0 else 0.0
    return max(FLOOR, float(np.log10(err))) if err > 0 else FLOOR


def features(order, nguard, cdt_dx, lam_dx, width, steps):
    """The six network inputs: 2/p (0 for infinite order), log2 n_g, c dt/dx, lambda/dx, 1/(k0 L), log2 steps."""
    order = np.asarray(order, dtype=np.float64)
    inv_p = np.where(order > 0, 2.0 / np.where(order > 0, order, 1.0), 0.0)
    return np.stack([inv_p, np.log2(np.asarray(nguard, dtype=np.float64)), np.asarray(cdt_dx, dtype=np.float64),
                     np.asarray(lam_dx, dtype=np.float64), np.asarray(width, dtype=np.float64),
                     np.log2(np.asarray(steps, dtype=np.float64))], axis=-1)
