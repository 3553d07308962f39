"""FP64 reference of the learned-initial-guess network (oracle; test-only).

Not part of the paper: the network is an addition that supplies U_0.
Architecture: five 3x3 cross-correlation layers with zero "same" padding,
channels 2 -> 32 -> 32 -> 32 -> 32 -> 1, exact GELU
x * Phi(x) = x (1 + erf(x / sqrt 2)) / 2 after layers 1-4.  Input channels:
f / 50 and v0 = A_h^-1 f (one tensor-product solve of the source); output: g,
a prediction of the pointwise nonlinear term U*^3, from which the caller forms
U_0 = A_h^-1 (f - g).  Loss = mean squared error; optimiser = Adam
(Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Arrays are NCHW.  Parameters are a flat vector in the order
W1 (32,2,3,3), b1 (32), W2, b2, W3, b3, W4, b4 (32,32,3,3)+(32), W5 (1,32,3,3), b5 (1),
weights indexed (out channel, in channel, dy, dx).  Pinned by finite differences
and a hand-computed single-layer example (tests/test_oracle_net.py).
"""

import math

import numpy as np

CHANNELS = (2, 32, 32, 32, 32, 1)
INPUT_SCALE = 1.0 / 50.0


def layer_shapes():
    out = []
    for i in range(5):
        cin, cout = CHANNELS[i], CHANNELS[i + 1]
        out.append(((cout, cin, 3, 3), (cout,)))
    return out


def param_count():
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in layer_shapes())


def unpack(theta):
    layers, o = [], 0
    for ws, bs in layer_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        layers.append((theta[o:o + nw].reshape(ws), theta[o + nw:o + nw + nb]))
        o += nw + nb
    return layers


def pack(layers):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in layers])


def he_init(seed=0):
    """He-normal weights (std sqrt(2 / fan_in), fan_in = 9 * c_in), zero biases."""
    rng = np.random.default_rng(seed)
    layers = []
    for ws, bs in layer_shapes():
        std = math.sqrt(2.0 / (ws[1] * 9))
        layers.append((rng.standard_normal(ws) * std, np.zeros(bs)))
    return pack(layers)


def conv3x3(a, w, b):
    """z[n, o, y, x] = b[o] + sum_{c, dy, dx} w[o, c, dy, dx] a[n, c, y+dy-1, x+dx-1],
    zero outside the image."""
    n, c, h, wd = a.shape
    ap = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1)))
    z = np.zeros((n, w.shape[0], h, wd)) + b[None, :, None, None]
    for dy in range(3):
        for dx in range(3):
            patch = ap[:, :, dy:dy + h, dx:dx + wd]
            z += np.einsum("oc,nchw->nohw", w[:, :, dy, dx], patch)
    return z


def conv3x3_loops(a, w, b):
    """Same as conv3x3 by scalar loops (tiny sizes only; pins conv3x3)."""
    n, c, h, wd = a.shape
    o = w.shape[0]
    z = np.zeros((n, o, h, wd))
    for i in range(n):
        for oc in range(o):
            for y in range(h):
                for x in range(wd):
                    s = b[oc]
                    for ic in range(c):
                        for dy in range(3):
                            for dx in range(3):
                                yy, xx = y + dy - 1, x + dx - 1
                                if 0 <= yy < h and 0 <= xx < wd:
                                    s += w[oc, ic, dy, dx] * a[i, ic, yy, xx]
                    z[i, oc, y, x] = s
    return z


_erf = np.vectorize(math.erf)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + _erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def features(f, v0):
    """Network input (N, 2, H, W) from the source f and v0 = A_h^-1 f."""
    return np.stack([f * INPUT_SCALE, v0], axis=1)


def forward(theta, x):
    """x: (N, 2, H, W) input features.  Returns (output (N, H, W), cache)."""
    layers = unpack(theta)
    a = np.asarray(x, dtype=np.float64)
    cache = {"a0": a, "z": []}
    for li, (w, b) in enumerate(layers):
        z = conv3x3(a, w, b)
        cache["z"].append(z)
        a = gelu(z) if li < 4 else z
        cache[f"a{li + 1}"] = a
    return a[:, 0], cache


def mse(pred, target):
    return float(np.mean((pred - target) ** 2))


def conv3x3_grads(a, w, dz):
    """Gradients of z = conv3x3(a, w, b) given dL/dz: returns (dw, db, da)."""
    n, c, h, wd = a.shape
    ap = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dap = np.zeros_like(ap)
    dw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            patch = ap[:, :, dy:dy + h, dx:dx + wd]
            dw[:, :, dy, dx] = np.einsum("nohw,nchw->oc", dz, patch)
            dap[:, :, dy:dy + h, dx:dx + wd] += np.einsum("oc,nohw->nchw", w[:, :, dy, dx], dz)
    db = dz.sum(axis=(0, 2, 3))
    return dw, db, dap[:, :, 1:-1, 1:-1]


def loss_and_grad(theta, x, target):
    """MSE loss of forward(theta, x) against target and its gradient (flat)."""
    layers = unpack(theta)
    pred, cache = forward(theta, x)
    loss = mse(pred, target)
    dz = (2.0 / pred.size) * (pred - target)[:, None]
    grads = [None] * 5
    for li in range(4, -1, -1):
        a_in = cache[f"a{li}"]
        dw, db, da = conv3x3_grads(a_in, layers[li][0], dz)
        grads[li] = (dw, db)
        if li > 0:
            dz = da * gelu_grad(cache["z"][li - 1])
    return loss, pack(grads)


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
