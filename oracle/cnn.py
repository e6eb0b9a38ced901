"""FP64 oracle of the learned force closure (TEST INFRASTRUCTURE).

The closure is not part of the paper's method: it is a small 3D convolutional
network that predicts, from fields on the 1x mesh, the difference between the
gathered force of a 2x-resolution mesh and of the 1x mesh.  Architecture:
conv(4 -> 16) - ReLU - conv(16 -> 16) - ReLU - conv(16 -> 3), 3x3x3 kernels,
periodic padding, cross-correlation taps d in {-1, 0, 1}^3:

    y[co, p] = b[co] + sum_{ci, d} W[co, ci, d] x[ci, p + d].

Mixed precision of the GPU path, emulated here: inputs, weights and the two
hidden activations are rounded to bfloat16 (round to nearest, ties to even)
where the GPU stores them; sums are exact (FP64).

Also: CIC gather of a vector field at particles and its adjoint (the deposit),
the closure's input features, the particle MSE and its gradient, the cube
symmetries used to augment training data and the Adam update.

Fields are arrays [c][z][y][x]; parameters use one flat FP32 vector with the
layout W1[16][4][27] b1[16] W2[16][16][27] b2[16] W3[3][16][27] b3[3], tap
index t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1).
"""
from __future__ import annotations

import numpy as np

from .pm import _corners, grad

LAYERS = ((4, 16), (16, 16), (16, 3))
N_PARAMS = sum(co * ci * 27 + co for ci, co in LAYERS)
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), f.astype(np.float64), out)


def unpack(params: np.ndarray):
    """Flat parameter vector -> [(W (co, ci, 27), b (co,)) per layer]."""
    out, o = [], 0
    for ci, co in LAYERS:
        w = params[o:o + co * ci * 27].reshape(co, ci, 27)
        o += co * ci * 27
        b = params[o:o + co]
        o += co
        out.append((np.asarray(w, dtype=np.float64), np.asarray(b, dtype=np.float64)))
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([w.reshape(-1), b]) for w, b in layers])


def shift(x: np.ndarray, d) -> np.ndarray:
    """x[..., p + d] with periodic wrap for fields [c][z][y][x] and d = (dz, dy, dx)."""
    dz, dy, dx = d
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(-3, -2, -1))


def conv(x: np.ndarray, w: np.ndarray, b: np.ndarray | None) -> np.ndarray:
    """y[co] = b[co] + sum_{ci, t} w[co, ci, t] x[ci, p + d_t]."""
    co = w.shape[0]
    y = np.zeros((co,) + x.shape[1:])
    for t, d in enumerate(TAPS):
        xs = shift(x, d)
        y += np.einsum("oc,c...->o...", w[:, :, t], xs)
    if b is not None:
        y += b[:, None, None, None]
    return y


def conv_transpose(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of conv in x: dx[ci, p] = sum_{co, t} w[co, ci, t] dy[co, p - d_t]."""
    ci = w.shape[1]
    dx = np.zeros((ci,) + dy.shape[1:])
    for t, d in enumerate(TAPS):
        dys = shift(dy, tuple(-v for v in d))
        dx += np.einsum("oc,o...->c...", w[:, :, t], dys)
    return dx


def conv_weight_grad(x: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """dW[co, ci, t] = sum_p x[ci, p + d_t] dy[co, p]."""
    co, ci = dy.shape[0], x.shape[0]
    g = np.zeros((co, ci, 27))
    for t, d in enumerate(TAPS):
        g[:, :, t] = np.einsum("czyx,ozyx->oc", shift(x, d), dy)
    return g


def forward(params: np.ndarray, x: np.ndarray, emulate_bf16: bool = True):
    """Network output (3 channels, FP64) and the stored activations (as the GPU stores them)."""
    r = bf16_round if emulate_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    (w1, b1), (w2, b2), (w3, b3) = unpack(params)
    x0 = r(x)
    a1 = r(np.maximum(conv(x0, r(w1), b1), 0.0))
    a2 = r(np.maximum(conv(a1, r(w2), b2), 0.0))
    y = conv(a2, r(w3), b3)
    return y, (x0, a1, a2)


def backward(params: np.ndarray, acts, dy: np.ndarray, emulate_bf16: bool = True) -> np.ndarray:
    """Gradient of sum(dy * y) with respect to the flat parameters.

    With emulation, the incoming gradient and the back-propagated hidden
    gradients are rounded to bfloat16 where the GPU stores them.
    """
    r = bf16_round if emulate_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    (w1, b1), (w2, b2), (w3, b3) = unpack(params)
    x0, a1, a2 = acts
    d3 = r(dy)
    g3w, g3b = conv_weight_grad(a2, d3), d3.sum(axis=(1, 2, 3))
    d2 = r(conv_transpose(d3, r(w3)) * (a2 > 0))
    g2w, g2b = conv_weight_grad(a1, d2), d2.sum(axis=(1, 2, 3))
    d1 = r(conv_transpose(d2, r(w2)) * (a1 > 0))
    g1w, g1b = conv_weight_grad(x0, d1), d1.sum(axis=(1, 2, 3))
    return pack([(g1w, g1b), (g2w, g2b), (g3w, g3b)])


def gather(field: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """CIC interpolation of a [c][z][y][x] field at particle positions -> (N_p, c)."""
    n = field.shape[-1]
    flat = field.reshape(field.shape[0], -1)
    out = np.zeros((pos.shape[0], field.shape[0]))
    for idx, w in _corners(pos, n):
        out += w[:, None] * flat[:, idx].T
    return out


def gather_adjoint(vals: np.ndarray, pos: np.ndarray, n: int) -> np.ndarray:
    """Adjoint of gather: CIC deposit of per-particle vectors (N_p, c) -> [c][z][y][x]."""
    c = vals.shape[1]
    out = np.zeros((c, n ** 3))
    for idx, w in _corners(pos, n):
        for k in range(c):
            out[k] += np.bincount(idx, weights=w * vals[:, k], minlength=n ** 3)
    return out.reshape(c, n, n, n)


def features(n00: np.ndarray, phi: np.ndarray):
    """Closure inputs: sign(delta) log(1 + |delta|) and grad phi / rms|grad phi|; returns (x, rms)."""
    n = n00.shape[-1]
    delta = n00 / n00.mean() - 1.0
    g = grad(phi, n)
    rms = float(np.sqrt(np.mean(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)))
    x = np.stack([np.sign(delta) * np.log1p(np.abs(delta)), g[0] / rms, g[1] / rms, g[2] / rms])
    return x, rms


def mse_loss(pred: np.ndarray, target: np.ndarray):
    """Particle mean-squared error over all components and its gradient in pred:
    (mean |pred - target|^2, mean |target|^2, 2 (pred - target) / numel)."""
    r = np.asarray(pred, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    return float(np.mean(r * r)), float(np.mean(t * t)), 2.0 * r / r.size


def cube_symmetry(pos: np.ndarray, u: np.ndarray, v: np.ndarray, perm, flip: int):
    """One of the 48 symmetries of the periodic unit cube on particle data [n][3]: component d of the
    result is component perm[d] of the input; where bit d of flip is set the position is reflected
    (x -> 1 - x, taken back into [0, 1)) and the two vector fields are negated."""
    perm = list(perm)
    p, a, b = pos[:, perm].copy(), u[:, perm].copy(), v[:, perm].copy()
    for d in range(3):
        if (flip >> d) & 1:
            x = 1.0 - p[:, d]
            p[:, d] = np.where(x >= 1.0, x - 1.0, x)
            a[:, d] = -a[:, d]
            b[:, d] = -b[:, d]
    return p, a, b


def adam(params, m, v, g, step: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (bias-corrected); returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
