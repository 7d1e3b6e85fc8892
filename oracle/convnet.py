"""Three-layer 3-D convolutional preconditioner: plain FP64 reference.  TEST INFRASTRUCTURE ONLY.

Not from the paper (which uses the eigensolvers' own preconditioners, Sec. 3.1): a learned map
from an eigensolver residual to a correction, x -> conv(8) -> ReLU -> conv(8) -> ReLU -> conv(1),
3x3x3 kernels, zero padding, one input and one output channel.  Written from the definition:

    y[o](p) = b[o] + sum_i sum_{d in {-1,0,1}^3} w[o, i, d + 1](p + d) x[i](p + d)    (zero outside)

and its exact gradients for the loss L = 1/2 sum (y - t)^2 / count.

Pinned by tests/test_oracle_scf.py: a delta input reproduces the (flipped) kernel, equality
with scipy.ndimage.correlate, and the analytic gradients against central finite differences.
"""

import numpy as np

LAYERS = ((1, 8), (8, 8), (8, 1))  # (input channels, output channels)
OFFSETS = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)]


def shifted(x, d):
    """s(p) = x(p + d) with zeros outside the box; x: (..., n, n, n)."""
    out = np.zeros_like(x)
    n = x.shape[-1]
    src = tuple(slice(max(0, k), n + min(0, k)) for k in d)
    dst = tuple(slice(max(0, -k), n - max(0, k)) for k in d)
    out[(Ellipsis,) + dst] = x[(Ellipsis,) + src]
    return out


def conv3d(x, w, b):
    """x: (Cin, n, n, n), w: (Cout, Cin, 3, 3, 3), b: (Cout,) -> (Cout, n, n, n)."""
    y = np.zeros((w.shape[0],) + x.shape[1:])
    y += b[:, None, None, None]
    for d in OFFSETS:
        xs = shifted(x, d)
        wd = w[:, :, d[0] + 1, d[1] + 1, d[2] + 1]
        y += np.tensordot(wd, xs, axes=(1, 0))
    return y


def forward(params, x):
    """params: list of (w, b); x: (n, n, n).  Returns (y (n, n, n), cache)."""
    a = x[None]
    cache = []
    for li, (w, b) in enumerate(params):
        z = conv3d(a, w, b)
        cache.append((a, z))
        a = np.maximum(z, 0.0) if li < len(params) - 1 else z
    return a[0], cache


def loss(y, t):
    return 0.5 * float(np.sum((y - t) ** 2)) / y.size


def backward(params, cache, y, t):
    """Gradients of loss(y, t) w.r.t. every (w, b)."""
    g = ((y - t) / y.size)[None]
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        w, b = params[li]
        a, z = cache[li]
        if li < len(params) - 1:
            g = g * (z > 0.0)
        gw = np.zeros_like(w)
        for d in OFFSETS:
            gw[:, :, d[0] + 1, d[1] + 1, d[2] + 1] = np.tensordot(g, shifted(a, d),
                                                                  axes=([1, 2, 3], [1, 2, 3]))
        gb = np.sum(g, axis=(1, 2, 3))
        grads[li] = (gw, gb)
        # gradient w.r.t. the layer input: sum_o sum_d w[o, i, d] g[o](p - d)
        ga = np.zeros_like(a)
        for d in OFFSETS:
            wd = w[:, :, d[0] + 1, d[1] + 1, d[2] + 1]
            ga += shifted(np.tensordot(wd, g, axes=(0, 0)), tuple(-k for k in d))
        g = ga
    return grads


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, bias-corrected moments) of a list of arrays, in place of
    copies: returns the new parameter list; ``state`` holds t and the moment arrays."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    if "m" not in state:
        state["m"] = [np.zeros_like(p) for p in params]
        state["v"] = [np.zeros_like(p) for p in params]
    out = []
    for i, (p, g) in enumerate(zip(params, grads)):
        state["m"][i] = b1 * state["m"][i] + (1.0 - b1) * g
        state["v"][i] = b2 * state["v"][i] + (1.0 - b2) * g * g
        mh = state["m"][i] / (1.0 - b1 ** t)
        vh = state["v"][i] / (1.0 - b2 ** t)
        out.append(p - lr * mh / (np.sqrt(vh) + eps))
    return out


def flatten(params):
    """Parameters as one vector in the order [w0, b0, w1, b1, w2, b2]."""
    return np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for w, b in params])


def unflatten(vec):
    out = []
    pos = 0
    for ci, co in LAYERS:
        nw = co * ci * 27
        w = np.asarray(vec[pos:pos + nw], dtype=np.float64).reshape(co, ci, 3, 3, 3)
        pos += nw
        b = np.asarray(vec[pos:pos + co], dtype=np.float64)
        pos += co
        out.append((w, b))
    return out


def init_params(rng, scale=0.2):
    return [(rng.normal(scale=scale / np.sqrt(27 * ci), size=(co, ci, 3, 3, 3)),
             np.zeros(co)) for ci, co in LAYERS]
