"""FP64 oracle of the warm-start network (TEST INFRASTRUCTURE ONLY).

Used by the tests to check the HIP inference/training kernels; shares no
code with them.  Plain numpy: each 3x3x3 convolution is written as the sum
over its 27 taps of a channel contraction of the shifted input.

Network (learned warm start of the Q field around a colloid in a
cholesteric; not part of the paper's method, whose plain relaxation stays
the judge of the prediction):
  features (12 channels) -> conv 12->32, SiLU -> conv 32->32, SiLU
  -> conv 32->32, SiLU -> conv 32->5 (linear) = dQ
  Q_warm = Q_helix + q_eq * dQ
A convolution with periodic padding:
  y[o](p) = b[o] + sum_c sum_t W[o, c, t] x[c](p + d_t),
  tap t = (dz+1)*9 + (dy+1)*3 + (dx+1), d_t = (dx, dy, dz) in {-1,0,1}^3.
Loss: mean over fluid sites of |Q_warm - Q_target|_F^2 (full 3x3 norm of the
traceless symmetric tensor stored as xx, xy, xz, yy, yz).
BF16 mode: weights and every layer input are rounded to bfloat16 (round to
nearest even) before the contraction; accumulation stays FP64.
"""
import math

import numpy as np

CHANNELS = (12, 32, 32, 32, 5)
TAPS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even) via float32; returns float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shift(x, d):
    """x shifted so that out[..., p] = x[..., p + d] (periodic), d = (dx, dy, dz)."""
    dx, dy, dz = d
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(-3, -2, -1))


def conv3d(x, W, b):
    """x (C, Z, Y, X), W (O, C, 27), b (O,) -> (O, Z, Y, X).

    Per tap, the channel contraction is a matrix product of W[:, :, t]
    (O x C) with the shifted input seen as C x sites."""
    C = x.shape[0]
    Wt = np.ascontiguousarray(W.transpose(2, 0, 1))   # (27, O, C)
    y = np.zeros((W.shape[0], x[0].size))
    for t, d in enumerate(TAPS):
        y += Wt[t] @ shift(x, d).reshape(C, -1)
    return y.reshape((W.shape[0],) + x.shape[1:]) + b[:, None, None, None]


def conv3d_backward(x, W, dy):
    """Gradients of sum(dy * conv3d(x, W, b)) with respect to x, W and b."""
    C, O = x.shape[0], dy.shape[0]
    dW = np.zeros_like(W)
    dx = np.zeros((C, x[0].size))
    g = dy.reshape(O, -1)
    WT = np.ascontiguousarray(W.transpose(2, 1, 0))   # (27, C, O)
    for t, d in enumerate(TAPS):
        dW[:, :, t] = g @ shift(x, d).reshape(C, -1).T
        dx += WT[t] @ shift(dy, (-d[0], -d[1], -d[2])).reshape(O, -1)
    return dx.reshape(x.shape), dW, dy.sum(axis=(1, 2, 3))


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def init_params(seed, channels=CHANNELS):
    """He-style uniform init from a seeded generator: W ~ U(-s, s), s = sqrt(6 / (27 C_in)); b = 0."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        s = math.sqrt(6.0 / (27 * cin))
        params.append((rng.uniform(-s, s, size=(cout, cin, 27)), np.zeros(cout)))
    return params


def forward(params, x, bf16=False):
    """Returns the output and the cache of (layer input, pre-activation)."""
    cache = []
    h = x
    n = len(params)
    for l, (W, b) in enumerate(params):
        xin = bf16_round(h) if bf16 else h
        Wl = bf16_round(W) if bf16 else W
        z = conv3d(xin, Wl, b)
        cache.append((xin, Wl, z))
        h = silu(z) if l < n - 1 else z
    return h, cache


def q_norm2(d):
    """Full-tensor |A|^2 of a traceless symmetric tensor field (5, ...)."""
    xx, xy, xz, yy, yz = d
    return 2 * (xx * xx + yy * yy + xx * yy + xy * xy + xz * xz + yz * yz)


def loss_and_grad(dq, q_helix, q_target, fluid, q_eq):
    """Loss and its gradient with respect to dq (5, Z, Y, X)."""
    d = q_helix + q_eq * dq - q_target
    nf = fluid.sum()
    loss = float((q_norm2(d) * fluid).sum() / nf)
    xx, xy, xz, yy, yz = d
    g = np.stack([4 * xx + 2 * yy, 4 * xy, 4 * xz, 4 * yy + 2 * xx, 4 * yz]) * fluid * (q_eq / nf)
    return loss, g


def backward(params, cache, dout, bf16=False):
    """Gradients of the loss for each layer given d(loss)/d(output).

    In BF16 mode the gradient entering each convolution is rounded to
    bfloat16 as well (the GPU feeds it to the matrix cores)."""
    grads = [None] * len(params)
    g = dout
    for l in range(len(params) - 1, -1, -1):
        xin, Wl, z = cache[l]
        if l < len(params) - 1:
            g = g * silu_grad(z)
        gin = bf16_round(g) if bf16 else g
        dx, dW, db = conv3d_backward(xin, Wl, gin)
        grads[l] = (dW, db)
        g = dx
    return grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (in place on copies); state = (t, m list, v list)."""
    t, ms, vs = state
    t += 1
    out, nm, nv = [], [], []
    for (W, b), (dW, db), (mW, mb), (vW, vb) in zip(params, grads, ms, vs):
        new = []
        for p, g, m, v in ((W, dW, mW, vW), (b, db, mb, vb)):
            m = beta1 * m + (1 - beta1) * g
            v = beta2 * v + (1 - beta2) * g * g
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            new.append((p - lr * mh / (np.sqrt(vh) + eps), m, v))
        out.append((new[0][0], new[1][0]))
        nm.append((new[0][1], new[1][1]))
        nv.append((new[0][2], new[1][2]))
    return out, (t, nm, nv)


def adam_init(params):
    z = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    return (0, z, [(np.zeros_like(W), np.zeros_like(b)) for W, b in params])


def features(L, pos, a, pitch, anchoring_sign, q_helix_unit):
    """12 input channels on an L^3 periodic grid (x fastest).

    0: clip((|x - R| - a)/8, -1, 2); 1-3: unit vector from the centre;
    4-8: helix Q divided by its amplitude; 9: a/16; 10: 32/pitch;
    11: +1 homeotropic, -1 planar anchoring.
    """
    g = np.arange(L, dtype=np.float64)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    r = [x - pos[0], y - pos[1], z - pos[2]]
    r = [np.where(v > L / 2, v - L, np.where(v < -L / 2, v + L, v)) for v in r]
    rn = np.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2)
    safe = np.where(rn > 0, rn, 1.0)
    f = np.zeros((12, L, L, L))
    f[0] = np.clip((rn - a) / 8.0, -1.0, 2.0)
    for k in range(3):
        f[1 + k] = np.where(rn > 0, r[k] / safe, 0.0)
    f[4:9] = q_helix_unit
    f[9] = a / 16.0
    f[10] = 32.0 / pitch
    f[11] = anchoring_sign
    return f
