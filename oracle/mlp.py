"""FP64 reference of the learned Newton initial guess (test infrastructure).

A 3-64-64-1 perceptron with SiLU activations predicts the standardised log of the Newton unknown
ht of Eq. 15 from three log-scaled invariants of the conserved state:
    f = (log D, log max(|M|/D, 1e-300), log(Et/D)),   x = (f - mean_in) / std_in,
    a1 = W1 x + b1,  h1 = SiLU(a1),  a2 = W2 h1 + b2,  h2 = SiLU(a2),  z = W3 h2 + b3,
    log ht_guess = mean_out + std_out * z,
with SiLU(a) = a / (1 + e^-a).  The GPU kernel keeps the weights in BF16 and feeds h1 to the
matrix cores in BF16 (FP32 accumulation); with ``bf16=True`` this reference applies exactly those
two roundings (round-to-nearest-even) and computes everything else in FP64.

The loss is the mean squared error of z against the standardised target; the gradient is written
out by hand (the backward treats the BF16 rounding of h1 as the identity).  Adam follows Kingma &
Ba (2015).  Parameter vector layout (4481 values): W1[64][3], b1[64], W2[64][64], b2[64],
W3[64], b3.
"""
import numpy as np

H = 64
SIZES = (("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,)))
N_PARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(a32), np.nan, out)


def silu(a):
    return a / (1.0 + np.exp(-a))


def dsilu(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def features(cons, kind=0):
    """cons [5][n] (D, Mx, My, Mz, Et) -> raw features [3][n]: kind 0 (log D, log max(|M|/D,
    1e-300), log(Et/D)); kind 1 the same with log L first, L of Eq. 15 correctly rounded (the
    oracle's), 0 for states that are not admissible (Eq. 30)."""
    cons = np.asarray(cons, dtype=np.float64)
    D = cons[0]
    m = np.sqrt((cons[1:4] ** 2).sum(axis=0)) / D
    if kind == 1:
        from oracle import L_batch
        L = L_batch(cons)
        ok = (D > 0) & (cons[4] > 0) & np.isfinite(L) & (L > np.finfo(np.float64).eps)
        with np.errstate(divide="ignore"):
            first = np.log(np.where(ok, L, 0.0))
    else:
        first = np.log(D)
    with np.errstate(divide="ignore", invalid="ignore"):     # unphysical inputs give NaN features
        return np.stack([first, np.log(np.maximum(m, 1e-300)), np.log(cons[4] / D)])


def forward(theta, x, bf16_round=True):
    """Standardised inputs x [3][n] -> (z [n], cache)."""
    p = unpack(theta)
    W1, W2, W3 = p["W1"], p["W2"], p["W3"]
    if bf16_round:
        W1, W2, W3 = bf16(W1), bf16(W2), bf16(W3)
    a1 = W1 @ x + p["b1"][:, None]
    h1 = silu(a1)
    h1m = bf16(h1) if bf16_round else h1
    a2 = W2 @ h1m + p["b2"][:, None]
    h2 = silu(a2)
    z = W3 @ h2 + p["b3"][0]
    return z, dict(x=x, a1=a1, h1m=h1m, a2=a2, h2=h2, W1=W1, W2=W2, W3=W3)


def loss_and_grad(theta, x, t, bf16_round=True):
    """Mean squared error of z against targets t [n] and its gradient (flat, N_PARAM)."""
    z, c = forward(theta, x, bf16_round)
    n = x.shape[1]
    r = z - t
    loss = float(np.mean(r * r))
    dz = 2.0 * r / n                                   # [n]
    g = {}
    g["W3"] = c["h2"] @ dz
    g["b3"] = np.array([dz.sum()])
    da2 = (c["W3"][:, None] * dz[None, :]) * dsilu(c["a2"])     # [H][n]
    g["W2"] = da2 @ c["h1m"].T
    g["b2"] = da2.sum(axis=1)
    da1 = (c["W2"].T @ da2) * dsilu(c["a1"])
    g["W1"] = da1 @ x.T
    g["b1"] = da1.sum(axis=1)
    return loss, pack(g)


def adam(theta, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init(seed=0):
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SIZES:
        if name.startswith("W"):
            fan_in = shape[1] if len(shape) == 2 else shape[0]
            fan_out = shape[0] if len(shape) == 2 else 1
            lim = np.sqrt(6.0 / (fan_in + fan_out))
            p[name] = rng.uniform(-lim, lim, size=shape)
        else:
            p[name] = np.zeros(shape)
    return pack(p)
