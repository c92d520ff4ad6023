"""FP64 reference of the learned warm start's network (test infrastructure only).

A U-Net on periodic lattice fields: 3x3 convolutions with circular padding, ReLU,
2x2 max pooling, nearest 2x upsampling with channel concatenation of the skip
tensors, a 1x1 output head added to the input density channel (residual), mean
squared error and the Adam update (Kingma & Ba, 2015, Algorithm 1).  Tensors are
NHWC float64 arrays; convolution weights are [C_out, 3, 3, C_in] (tap (ky, kx)
reads the input at offset (ky-1, kx-1)).

Every operation is its plain definition, written out: convolutions as sums over
the nine taps of shifted copies (np.roll implements the periodic shift) times
the tap's weight matrix; gradients are the adjoint sums of the same terms.  The
tests pin them against finite differences, adjoint identities, a library
correlation and closed forms.

The GPU implementation shares nothing with this module.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# tap index t = (dy + 1) * 3 + (dx + 1) for the offset (dy, dx) read by the tap
TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shifted(x, dy, dx):
    """xs[n, y, x] = x[n, (y + dy) mod H, (x + dx) mod W]."""
    return np.roll(x, shift=(-dy, -dx), axis=(1, 2))


def conv3x3(x, w, b=None):
    """y[n,y,x,o] = b[o] + sum_{t,i} w[o,t,i] x[n, y+dy_t, x+dx_t, i] (periodic)."""
    co = w.shape[0]
    y = np.zeros(x.shape[:3] + (co,))
    for t, (dy, dx) in enumerate(TAPS):
        y += shifted(x, dy, dx) @ w[:, dy + 1, dx + 1, :].T
    if b is not None:
        y += b
    return y


def conv3x3_grad_input(g, w):
    """dL/dx for y = conv3x3(x, w): dx[p] = sum_t g[p - off_t] @ w_t."""
    ci = w.shape[3]
    dx_ = np.zeros(g.shape[:3] + (ci,))
    for dy, dx in TAPS:
        dx_ += shifted(g, -dy, -dx) @ w[:, dy + 1, dx + 1, :]
    return dx_


def conv3x3_grad_weight(x, g):
    """dL/dw[o,ky,kx,i] = sum_{n,p} g[n,p,o] x[n, p + off, i];  dL/db[o] = sum g[..., o]."""
    co, ci = g.shape[3], x.shape[3]
    dw = np.zeros((co, 3, 3, ci))
    g2 = g.reshape(-1, co)
    for dy, dx in TAPS:
        dw[:, dy + 1, dx + 1, :] = g2.T @ shifted(x, dy, dx).reshape(-1, ci)
    return dw, g2.sum(axis=0)


def relu(x):
    return np.maximum(x, 0.0)


def relu_grad(g, y):
    """Gradient through y = relu(z) given the output y (z > 0 exactly where y > 0)."""
    return g * (y > 0)


def maxpool2(x):
    """2x2 windows, stride 2 (H, W even)."""
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).max(axis=(2, 4))


def maxpool2_grad(x, g):
    """Routes each window's gradient to the first maximum in row-major window order
    ((0,0), (0,1), (1,0), (1,1))."""
    n, h, w, c = x.shape
    dx = np.zeros_like(x)
    taken = np.zeros(g.shape, dtype=bool)
    m = maxpool2(x)
    for a in (0, 1):
        for b in (0, 1):
            v = x[:, a::2, b::2, :]
            hit = (v == m) & ~taken
            dx[:, a::2, b::2, :] = np.where(hit, g, 0.0)
            taken |= hit
    return dx


def upsample2(x):
    """Nearest neighbour: y[n, 2y+a, 2x+b] = x[n, y, x]."""
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_grad(g):
    n, h, w, c = g.shape
    return g.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def head(d, w, b, rin):
    """out[n,y,x,k] = sum_c w[k,c] d[n,y,x,c] + b[k] + rin[n,y,x,k]: K outputs, each the
    residual on an input field (the density; with K = 2 also the temperature deviation)."""
    return d @ w.T + b + rin


def mse(pred, target):
    r = pred - target
    return float(np.mean(r * r)), 2.0 * r / r.size


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t >= 1), bias-corrected moments.  Returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------
@dataclass
class Arch:
    """Encoder widths per level (the bottleneck is the last); input channels (the first
    `used_inputs` carry data, the rest are zero padding)."""
    widths: tuple = (32, 64, 128, 256)
    in_channels: int = 8
    used_inputs: int = 3
    outputs: int = 1

    def residual_channels(self):
        """Input channels the head adds to its outputs: the density (channel 0) and, for a
        second output, the temperature deviation (channel 2)."""
        return [0, 2][: self.outputs]

    def convs(self):
        """(name, C_in, C_out) of every 3x3 convolution in order."""
        w = self.widths
        out = []
        cin = self.in_channels
        for lvl, c in enumerate(w):
            out += [(f"e{lvl}a", cin, c), (f"e{lvl}b", c, c)]
            cin = c
        for lvl in range(len(w) - 2, -1, -1):
            out += [(f"d{lvl}a", w[lvl + 1] + w[lvl], w[lvl]), (f"d{lvl}b", w[lvl], w[lvl])]
        return out


def init_params(arch: Arch, seed: int):
    """He-normal 3x3 weights (std sqrt(2 / (9 C_in))), zero biases, head weights
    N(0, 1/C) ([outputs, C]) and zero head biases; from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for name, ci, co in arch.convs():
        p[name + ".w"] = rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci))
        p[name + ".b"] = np.zeros(co)
    c0 = arch.widths[0]
    p["head.w"] = rng.standard_normal((arch.outputs, c0)) / np.sqrt(c0)
    p["head.b"] = np.zeros(arch.outputs)
    return p


def _exact(a):
    return a


def forward(arch: Arch, p: dict, x, store=_exact, rin=None):
    """x: [N, H, W, in_channels]; channel 0 is the normalised input density, channel 2
    the normalised temperature deviation.  Returns the prediction [N, H, W, outputs]
    and the activations the backward pass needs.

    store: applied to every convolution output (identity by default; bf16_round
    models an implementation that keeps activations in bfloat16).  rin: the fields
    the head adds ([N, H, W, outputs]; default the residual channels of x)."""
    cache = {"x": x}
    h = x
    skips = []
    L = len(arch.widths)
    for lvl in range(L):
        a = store(relu(conv3x3(h, p[f"e{lvl}a.w"], p[f"e{lvl}a.b"])))
        bb = store(relu(conv3x3(a, p[f"e{lvl}b.w"], p[f"e{lvl}b.b"])))
        cache[f"e{lvl}_in"], cache[f"e{lvl}a"], cache[f"e{lvl}b"] = h, a, bb
        if lvl < L - 1:
            skips.append(bb)
            h = maxpool2(bb)
        else:
            h = bb
    for lvl in range(L - 2, -1, -1):
        cat = np.concatenate([upsample2(h), skips[lvl]], axis=3)
        a = store(relu(conv3x3(cat, p[f"d{lvl}a.w"], p[f"d{lvl}a.b"])))
        bb = store(relu(conv3x3(a, p[f"d{lvl}b.w"], p[f"d{lvl}b.b"])))
        cache[f"d{lvl}_in"], cache[f"d{lvl}a"], cache[f"d{lvl}b"] = cat, a, bb
        h = bb
    out = head(h, p["head.w"], p["head.b"], x[..., arch.residual_channels()] if rin is None else rin)
    return out, cache


def backward(arch: Arch, p: dict, cache: dict, dout, store=_exact):
    """Gradients of every parameter and of the input for dL/dout = dout.

    store: applied to every activation-gradient tensor an implementation would keep
    (ReLU-gated gradients of convolution outputs, input gradients of convolutions,
    the pooled-path gradients); identity by default."""
    gr = {}
    L = len(arch.widths)
    top = cache["d0b"]
    K = dout.shape[3]
    gr["head.w"] = dout.reshape(-1, K).T @ top.reshape(-1, top.shape[3])
    gr["head.b"] = dout.reshape(-1, K).sum(axis=0)
    dh = dout @ p["head.w"]
    dskip = {}
    # decoder levels ran L-2, ..., 0; their backward runs 0, ..., L-2
    for lvl in range(0, L - 1):
        gb = store(relu_grad(dh, cache[f"d{lvl}b"]))
        gr[f"d{lvl}b.w"], gr[f"d{lvl}b.b"] = conv3x3_grad_weight(cache[f"d{lvl}a"], gb)
        ga = store(relu_grad(conv3x3_grad_input(gb, p[f"d{lvl}b.w"]), cache[f"d{lvl}a"]))
        gr[f"d{lvl}a.w"], gr[f"d{lvl}a.b"] = conv3x3_grad_weight(cache[f"d{lvl}_in"], ga)
        dcat = store(conv3x3_grad_input(ga, p[f"d{lvl}a.w"]))
        cu = dcat.shape[3] - arch.widths[lvl]
        dskip[lvl] = dcat[..., cu:]
        dh = upsample2_grad(dcat[..., :cu])
    # encoder levels ran 0, ..., L-1; their backward runs L-1, ..., 0
    for lvl in range(L - 1, -1, -1):
        if lvl < L - 1:
            dh = maxpool2_grad(cache[f"e{lvl}b"], dh) + dskip[lvl]
        gb = store(relu_grad(dh, cache[f"e{lvl}b"]))
        gr[f"e{lvl}b.w"], gr[f"e{lvl}b.b"] = conv3x3_grad_weight(cache[f"e{lvl}a"], gb)
        ga = store(relu_grad(conv3x3_grad_input(gb, p[f"e{lvl}b.w"]), cache[f"e{lvl}a"]))
        gr[f"e{lvl}a.w"], gr[f"e{lvl}a.b"] = conv3x3_grad_weight(cache[f"e{lvl}_in"], ga)
        dh = conv3x3_grad_input(ga, p[f"e{lvl}a.w"])
        if lvl > 0:
            dh = store(dh)
    dx = dh.copy()
    for k, ch in enumerate(arch.residual_channels()):
        dx[..., ch] += dout[..., k]
    return gr, dx


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    return np.where(np.isfinite(a32), out, a32).astype(np.float64)
