"""Learned-gate MLP reference -- TEST INFRASTRUCTURE ONLY.

Plain numpy FP64 forward pass, mean-squared-error gradient and one Adam step
of the gate's cost model: 8 inputs -> 32 ReLU -> 32 ReLU -> 4 linear outputs,
parameters packed as W1[32x8] b1[32] W2[32x32] b2[32] W3[4x32] b3[4]
(row-major, out x in). Pinned in tests against central finite differences and
torch's CPU Linear/ReLU and Adam.
"""
import numpy as np

IN, HID, OUT = 8, 32, 4
SIZES = [(HID, IN), (HID,), (HID, HID), (HID,), (OUT, HID), (OUT,)]
NPARAMS = sum(int(np.prod(s)) for s in SIZES)


def unpack(p):
    p = np.asarray(p, np.float64)
    out, off = [], 0
    for s in SIZES:
        k = int(np.prod(s))
        out.append(p[off:off + k].reshape(s))
        off += k
    return out


def forward(p, x):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, np.float64)
    h1 = np.maximum(x @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ W3.T + b3


def loss(p, x, t, mask):
    """mean over samples of sum_j mask * (y - t)^2"""
    y = forward(p, x)
    e = (y - np.asarray(t, np.float64)) * np.asarray(mask, np.float64)
    return float((e * e).sum() / len(x))


def grad(p, x, t, mask):
    """Back-propagation of `loss` (chain rule through the two ReLU layers)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, np.float64)
    a1 = x @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ W3.T + b3
    n = len(x)
    dy = 2.0 * (y - t) * mask * mask / n
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dh2 = dy @ W3 * (a2 > 0)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(0)
    dh1 = dh2 @ W2 * (a1 > 0)
    gW1 = dh1.T @ x
    gb1 = dh1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam_step(p, g, m1, m2, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015); returns new (p, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, m2


def features(frontier, active, n, m, k, prev_us, prev_mode, app):
    """The gate's 8 input features (same definitions as the library header)."""
    return np.array([frontier / n, active / m, 1.0 - np.exp(-active / np.ceil(m / 16.0)),
                     app / 3.0, np.log2(m) / 32.0, min(k, 255) / 64.0,
                     np.log1p(prev_us) / 16.0, prev_mode / 3.0])
