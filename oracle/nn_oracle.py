"""FP64 reference of the surrogate network's building blocks.

TEST INFRASTRUCTURE. Only the test suite may import this module; the HIP
library and its Python package never do. Plain numpy, float64, written from
the definitions (no blocking, no fusion):

* circular 3x3 convolution y[b,y,x,o] = bias[o] +
  sum_{t,i} w[o,t,i] x[b,(y+dy_t) mod H,(x+dx_t) mod W,i],
  tap t = (dy+1)*3 + (dx+1);
* its data gradient and weight/bias gradients;
* 2x2 average pooling, nearest 2x upsampling and their adjoints;
* leaky ReLU (negative slope 1/8) and its derivative;
* the relative L2 loss (1/B) sum_b |p_b - t_b|^2 / |t_b|^2 and its gradient.

Layout: NHWC arrays (B, H, W, C); weights (C_out, 9, C_in).
"""
from __future__ import annotations

import numpy as np

SLOPE = 0.125
TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shift(x: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """s[b, y, x] = x[b, (y + dy) mod H, (x + dx) mod W]."""
    return np.roll(np.roll(x, -dy, axis=1), -dx, axis=2)


def conv3x3(x: np.ndarray, w: np.ndarray, bias=None) -> np.ndarray:
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    y = np.zeros(x.shape[:3] + (w.shape[0],))
    for t, (dy, dx) in enumerate(TAPS):
        y += shift(x, dy, dx) @ w[:, t, :].T
    if bias is not None:
        y += np.asarray(bias, np.float64)
    return y


def conv3x3_dgrad(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """dL/dx for y = conv3x3(x, w): the input value at p + offset(t) met
    w[:, t, :] in the output at p, so it collects dy[p] w[:, t, :]."""
    dy = np.asarray(dy, np.float64)
    w = np.asarray(w, np.float64)
    dx = np.zeros(dy.shape[:3] + (w.shape[2],))
    for t, (sy, sx) in enumerate(TAPS):
        dx += shift(dy @ w[:, t, :], -sy, -sx)
    return dx


def conv3x3_wgrad(x: np.ndarray, dy: np.ndarray):
    """(dL/dw, dL/dbias) for y = conv3x3(x, w) + bias."""
    x = np.asarray(x, np.float64)
    dy = np.asarray(dy, np.float64)
    co, ci = dy.shape[3], x.shape[3]
    dw = np.zeros((co, 9, ci))
    g = dy.reshape(-1, co)
    for t, (sy, sx) in enumerate(TAPS):
        dw[:, t, :] = g.T @ shift(x, sy, sx).reshape(-1, ci)
    return dw, g.sum(axis=0)


def leaky(z: np.ndarray) -> np.ndarray:
    return np.where(z > 0, z, SLOPE * z)


def leaky_bwd(y: np.ndarray, dy: np.ndarray) -> np.ndarray:
    return np.where(y > 0, dy, SLOPE * dy)


def avgpool2(x: np.ndarray) -> np.ndarray:
    B, H, W, C = x.shape
    return np.asarray(x, np.float64).reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_bwd(dy: np.ndarray) -> np.ndarray:
    return 0.25 * np.repeat(np.repeat(np.asarray(dy, np.float64), 2, axis=1), 2, axis=2)


def upsample2(x: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(np.asarray(x, np.float64), 2, axis=1), 2, axis=2)


def upsample2_bwd(dy: np.ndarray) -> np.ndarray:
    B, H, W, C = dy.shape
    return np.asarray(dy, np.float64).reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def rel_l2(pred: np.ndarray, target: np.ndarray):
    """pred, target (B, ...): loss, per-sample relative error, gradient."""
    p = np.asarray(pred, np.float64)
    t = np.asarray(target, np.float64)
    B = p.shape[0]
    d = (p - t).reshape(B, -1)
    den = (t.reshape(B, -1) ** 2).sum(axis=1)
    num = (d ** 2).sum(axis=1)
    loss = float(np.mean(num / den))
    grad = (2.0 * d / (den[:, None] * B)).reshape(p.shape)
    return loss, np.sqrt(num / den), grad


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# The whole network (four-level U-net with additive skips), forward and
# backward, on a flat parameter vector laid out layer by layer as
# [w (c_out, 9, c_in) | bias (c_out)]. ``r`` rounds a stored activation
# (identity in exact FP64 mode, bf16_round to mirror BF16 storage).
# ---------------------------------------------------------------------------

LEVELS = (32, 64, 128, 128)
BOTTLENECK = 4
IN_CH, OUT_CH = 48, 32


def unet_layers():
    """(name, c_in, c_out, leaky, level) in parameter order."""
    out = [("e0a", IN_CH, 32, True, 0), ("e0", 32, 32, True, 0)]
    for l in (1, 2, 3):
        out += [(f"e{l}a", LEVELS[l - 1], LEVELS[l], True, l), (f"e{l}", LEVELS[l], LEVELS[l], True, l)]
    out += [(f"b{k}", 128, 128, True, 4) for k in range(BOTTLENECK)]
    prev = LEVELS[3]
    for l in (3, 2, 1, 0):
        out += [(f"d{l}a", prev, LEVELS[l], True, l), (f"d{l}", LEVELS[l], LEVELS[l], True, l)]
        prev = LEVELS[l]
    out.append(("out", 32, OUT_CH, False, 0))
    return out


def unpack_params(p):
    views, off = {}, 0
    for name, ci, co, _, _ in unet_layers():
        nw = co * 9 * ci
        views[name] = (np.asarray(p[off:off + nw], np.float64).reshape(co, 9, ci),
                       np.asarray(p[off + nw:off + nw + co], np.float64))
        off += nw + co
    return views, off


def unet_forward(p, x, bf16=False):
    """x (B, H, W, 16); returns (out (B, H, W, 32) FP64, saved activations)."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    P, _ = unpack_params(p)
    wq = {k: (r(w) if bf16 else w, b) for k, (w, b) in P.items()}
    act = {"x": r(x)}

    def layer(name, inp, leaky_on=True):
        w, b = wq[name]
        z = conv3x3(inp, w, b)
        y = r(leaky(z)) if leaky_on else z
        act[name] = y
        return y

    h = act["x"]
    for l in range(4):
        if l:
            h = r(avgpool2(h))
            act[f"p{l}"] = h
        h = layer(f"e{l}a", h)
        h = layer(f"e{l}", h)
    h = r(avgpool2(h))
    act["p4"] = h
    for k in range(BOTTLENECK):
        h = layer(f"b{k}", h)
    for l in (3, 2, 1, 0):
        u = upsample2(h)
        act[f"u{l}"] = u
        d = layer(f"d{l}a", u)
        hh = r(d + act[f"e{l}"])
        act[f"h{l}"] = hh
        h = layer(f"d{l}", hh)
    out = layer("out", h, leaky_on=False)
    return out, act


def unet_backward(p, act, dout, bf16=False):
    """Gradient of the flat parameters given dL/dout, on the saved
    activations; with bf16=True every stored activation gradient is rounded
    to bfloat16 where a BF16 implementation stores it."""
    r = bf16_round if bf16 else (lambda a: a)
    P, n = unpack_params(p)
    grads = {}

    def back(name, inp, dy, leaky_on=True, need_dx=True):
        w, _ = P[name]
        dz = r(leaky_bwd(act[name], dy)) if leaky_on else dy
        grads[name] = conv3x3_wgrad(inp, dz)
        act["dz_" + name] = dz
        dx = r(conv3x3_dgrad(dz, w)) if need_dx else None
        act["dx_" + name] = dx
        return dx

    g = back("out", act["d0"], dout, leaky_on=False)
    for l in (0, 1, 2, 3):
        gh = back(f"d{l}", act[f"h{l}"], g)
        act[f"gh{l}"] = gh
        gu = back(f"d{l}a", act[f"u{l}"], gh)
        g = r(upsample2_bwd(gu))
    for k in range(BOTTLENECK - 1, -1, -1):
        inp = act["p4"] if k == 0 else act[f"b{k - 1}"]
        g = back(f"b{k}", inp, g)
    for l in (3, 2, 1, 0):
        ge = r(act[f"gh{l}"] + avgpool2_bwd(g))
        ga = back(f"e{l}", act[f"e{l}a"], ge)
        inp = act["x"] if l == 0 else act[f"p{l}"]
        g = back(f"e{l}a", inp, ga, need_dx=l > 0)
    flat = np.zeros(n)
    off = 0
    for name, ci, co, _, _ in unet_layers():
        dw, db = grads[name]
        flat[off:off + co * 9 * ci] = dw.ravel()
        flat[off + co * 9 * ci:off + co * 9 * ci + co] = db
        off += co * 9 * ci + co
    return flat
