"""FP64 reference of the surrogate MLP 4-128-128-3 -- TEST INFRASTRUCTURE ONLY.

Mirrors the BF16 rounding points of the HIP kernels (weights and the
activations that enter matrix products are rounded FP32 -> BF16, round to
nearest even), with every sum in FP64:

  forward : xb = bf16(x); z1 = W1b xb + b1; h1 = bf16(silu z1);
            z2 = W2b h1 + b2; h2 = bf16(silu z2); y = W3b h2 + b3
  backward: dY = 2 w (y - t) / B;  dW3 = dY^T h2; dH2 = dY W3b;
            dz2 = dH2 silu'(z2); dz2b = bf16(dz2);
            dW2 = dz2b^T h1; dH1 = dz2b W2b; dz1 = dH1 silu'(z1);
            dW1 = dz1^T xb; dx = dz1 W1b; bias gradients sum the unrounded dz.
  Adam    : the update of Kingma & Ba with bias correction (the optimiser the
            paper uses for its optimisation experiments, Results).

Parameter layout (one flat vector): W1[128][4], b1[128], W2[128][128],
b2[128], W3[3][128], b3[3].

Pins (tests/test_oracle_mlp.py): bf16() against torch's float32 -> bfloat16
conversion; with rounding disabled, forward and backward against torch
autograd in FP64; Adam against torch.optim.Adam in FP64.
"""
import numpy as np

IN, H, OUT = 4, 128, 3
SHAPES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (OUT, H)),
          ("b3", (OUT,))]
NP = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16(x):
    """Round to the nearest BF16 (ties to even) through FP32; returns FP64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(P):
    P = np.asarray(P, np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = P[o:o + n].reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in SHAPES])


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def init_params(rng):
    """He-style uniform initialisation (FP32 values)."""
    d = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shp[1])
            d[name] = rng.uniform(-bound, bound, size=shp)
        else:
            d[name] = np.zeros(shp)
    return pack(d).astype(np.float32)


def forward(P, x, rounding=True):
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    p = unpack(P)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    xb = r(x)
    z1 = xb @ W1.T + p["b1"]
    h1 = r(silu(z1))
    z2 = h1 @ W2.T + p["b2"]
    h2 = r(silu(z2))
    y = h2 @ W3.T + p["b3"]
    return y, dict(xb=xb, z1=z1, h1=h1, z2=z2, h2=h2, W1=W1, W2=W2, W3=W3)


def backward(P, x, t, w, rounding=True):
    """Returns (grad[NP], dx[B, 4], loss) of L = mean_b sum_j w_j (y - t)^2."""
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    y, c = forward(P, x, rounding)
    B = y.shape[0]
    w = np.asarray(w, np.float64)
    e = y - np.asarray(t, np.float64)
    loss = float(np.sum(w * e * e) / B)
    dY = 2.0 * w * e / B
    g = {}
    g["W3"] = dY.T @ c["h2"]
    g["b3"] = dY.sum(axis=0)
    dH2 = dY @ c["W3"]
    dz2 = dH2 * dsilu(c["z2"])
    dz2b = r(dz2)
    g["W2"] = dz2b.T @ c["h1"]
    g["b2"] = dz2.sum(axis=0)
    dH1 = dz2b @ c["W2"]
    dz1 = dH1 * dsilu(c["z1"])
    g["W1"] = dz1.T @ c["xb"]
    g["b1"] = dz1.sum(axis=0)
    dx = dz1 @ c["W1"]
    return pack(g), dx, loss


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected moments); returns new (p, m, v)."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def magnitude_bounds(P, x, t, w):
    """|.|-propagated magnitudes of every output of forward/backward (the same
    products with absolute values of every factor), used to scale the
    tolerance of a comparison: a BF16 rounding decision taken from an FP32
    instead of an FP64 sum moves a rounded value by one BF16 step (2^-8
    relative), so the deviation of each result is a small multiple of 2^-8
    times its magnitude bound.  Returns (|y|, |grad|, |dx|)."""
    p = unpack(P)
    W1, W2, W3 = (np.abs(bf16(p[k])) for k in ("W1", "W2", "W3"))
    y, c = forward(P, x, True)
    B = y.shape[0]
    ax = np.abs(c["xb"])
    ah1, ah2 = np.abs(c["h1"]), np.abs(c["h2"])
    ay = ah2 @ W3.T + np.abs(p["b3"])
    e = np.abs(y - np.asarray(t, np.float64)) + ay
    adY = 2.0 * np.abs(w) * e / B
    g = {}
    g["W3"] = adY.T @ ah2
    g["b3"] = adY.sum(axis=0)
    dH2 = adY @ W3
    ds2 = np.abs(dsilu(c["z2"]))
    dz2 = dH2 * ds2
    g["W2"] = dz2.T @ ah1
    g["b2"] = dz2.sum(axis=0)
    dH1 = dz2 @ W2
    dz1 = dH1 * np.abs(dsilu(c["z1"]))
    g["W1"] = dz1.T @ ax
    g["b1"] = dz1.sum(axis=0)
    return ay, pack(g), dz1 @ W1
