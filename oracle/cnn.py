"""Plain FP64 convolutional network of the learned coarse-grid correction.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network is four 3x3 convolutions with circular (periodic) padding,
channels 3 -> 32 -> 32 -> 32 -> 3, ReLU after the first three:

    Y[b, co, y, x] = bias[co] + sum_{ci, dy, dx} W[co, ci, dy+1, dx+1] X[b, ci, y+dy, x+dx]

(indices mod H, W; a cross-correlation, as in common deep-learning
convention).  Forward, backward and Adam follow their textbook definitions;
a "library routine" cross-check is scipy.ndimage.correlate(mode="wrap").

Arrays: activations [B, C, H, W]; weights [Cout, Cin, 3, 3]; bias [Cout].
"""

from __future__ import annotations

import numpy as np

LAYERS = ((3, 32), (32, 32), (32, 32), (32, 3))
TAPS = tuple((dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1))


def shifted(x: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """s[..., y, x] = x[..., (y + dy) mod H, (x + dx) mod W]."""
    return np.roll(x, shift=(-dy, -dx), axis=(-2, -1))


def init_params(seed: int = 0, layers=LAYERS) -> list:
    """He-uniform weights, zero bias (a fixed, seeded starting point)."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in layers:
        bound = np.sqrt(6.0 / (cin * 9))
        w = rng.uniform(-bound, bound, (cout, cin, 3, 3))
        params.append((w, np.zeros(cout)))
    return params


def _ident(a):
    return a


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), as float64: the operand
    precision of a BF16 matrix multiply with FP32 accumulation."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv(x: np.ndarray, w: np.ndarray, b: np.ndarray | None, rnd=_ident) -> np.ndarray:
    x, w = rnd(x), rnd(w)
    bsz, cin, h, wd = x.shape
    cout = w.shape[0]
    y = np.zeros((bsz, cout, h, wd))
    for (dy, dx) in TAPS:
        xs = shifted(x, dy, dx)                            # [B, Cin, H, W]
        y += np.einsum("oc,bchw->bohw", w[:, :, dy + 1, dx + 1], xs)
    if b is not None:
        y += b[None, :, None, None]
    return y


def conv_backward(x: np.ndarray, w: np.ndarray, dy_: np.ndarray, rnd=_ident):
    """Gradients of Y = conv(X, W) + b given dL/dY: (dX, dW, db).  `rnd` is
    applied to the operands of the products (not to the bias sum)."""
    db = dy_.sum(axis=(0, 2, 3))
    x, w, dy_ = rnd(x), rnd(w), rnd(dy_)
    dw = np.zeros_like(w)
    dx_ = np.zeros_like(x)
    for (dy, dx) in TAPS:
        xs = shifted(x, dy, dx)
        dw[:, :, dy + 1, dx + 1] = np.einsum("bohw,bchw->oc", dy_, xs)
        # Y[y] gets W X[y + d]  =>  dX[z] += W^T dY[z - d]
        dx_ += np.einsum("oc,bohw->bchw", w[:, :, dy + 1, dx + 1], shifted(dy_, -dy, -dx))
    return dx_, dw, db


def forward(params: list, x: np.ndarray, rnd=_ident):
    """Returns (output, cache) with cache = list of (input, pre-activation) per layer."""
    cache = []
    a = x
    for li, (w, b) in enumerate(params):
        z = conv(a, w, b, rnd)
        cache.append((a, z))
        a = np.maximum(z, 0.0) if li < len(params) - 1 else z
    return a, cache


def backward(params: list, cache: list, dout: np.ndarray, rnd=_ident):
    """dL/dparams (list of (dW, db)) and dL/dx from dL/doutput."""
    grads = [None] * len(params)
    d = dout
    for li in range(len(params) - 1, -1, -1):
        a_in, z = cache[li]
        if li < len(params) - 1:
            d = d * (z > 0.0)
        dx_, dw, db = conv_backward(a_in, params[li][0], d, rnd)
        grads[li] = (dw, db)
        d = dx_
    return grads, d


def mse(out: np.ndarray, target: np.ndarray):
    """L = mean((out - target)^2) and dL/dout."""
    diff = out - target
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


class Adam:
    """Adam with bias correction (Kingma & Ba): m = b1 m + (1-b1) g,
    v = b2 v + (1-b2) g^2, p -= lr * m_hat / (sqrt(v_hat) + eps)."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
        self.v = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]

    def step(self, params, grads):
        self.t += 1
        out = []
        for i, ((w, b), (gw, gb)) in enumerate(zip(params, grads)):
            new = []
            for j, (p, g) in enumerate(((w, gw), (b, gb))):
                m = self.b1 * self.m[i][j] + (1 - self.b1) * g
                v = self.b2 * self.v[i][j] + (1 - self.b2) * g * g
                mh = m / (1 - self.b1 ** self.t)
                vh = v / (1 - self.b2 ** self.t)
                new.append(p - self.lr * mh / (np.sqrt(vh) + self.eps))
                if j == 0:
                    mw, vw = m, v
                else:
                    self.m[i] = (mw, m)
                    self.v[i] = (vw, v)
            out.append(tuple(new))
        return out
