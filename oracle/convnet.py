"""FP64 reference of the learned corrector's network, the box filter and the
field increments (test infrastructure: only tests/, the checker's smoke test
and the benchmark's CPU baseline use it; nothing here is shared with the HIP
library).

Network: layer l maps c[l] channels to c[l+1]:
    y[o](v) = b[o] + sum_t sum_i x[i](v + s_t) W[t][i][o],
s_t = (t%3 - 1, (t//3)%3 - 1, t//9 - 1) in (x, y, z), periodic; ReLU after
every layer but the last.  Arrays are [channel][z][y][x].  The training loss of
one sample is L = mean over nodes and channels of (y_c + (x_c - t_c)/s_c)^2
with y = network((x - mean)/std) and s the output scale (s = std unless given);
output c may belong to field c + offset (a network that corrects some of its
input fields).

Everything is written out with numpy in FP64; the backward pass follows the
chain rule layer by layer and is pinned by finite differences in the tests.

Optional storage rounding (store=bf16): the library keeps the network's
matrix-core operands in bfloat16 (normalised inputs, weights, hidden
activations, the loss gradient and the gradients passed between layers) and
accumulates in FP32.  With store=bf16 those values are rounded to bfloat16
where the library stores them, and everything else stays FP64, so the
comparison isolates what the format itself costs from accumulation order.
"""
from __future__ import annotations

import numpy as np

TAPS = [(t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1) for t in range(27)]


def shift(a, t, sign=1):
    """a moved so that out(v) = a(v + sign * s_t), periodic (last three axes z, y, x)."""
    dx, dy, dz = TAPS[t]
    return np.roll(a, shift=(-sign * dz, -sign * dy, -sign * dx), axis=(-3, -2, -1))


def bf16(a):
    """Round to the nearest bfloat16 (1 sign, 8 exponent, 7 fraction bits),
    ties to even, via the FP32 bit pattern (the value is first rounded to
    FP32); returned as FP64."""
    a = np.asarray(a, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    keep = (bits >> 16) & 1  # lowest kept bit: ties go to the even neighbour
    r = ((bits + 0x7FFF + keep) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _same(a):
    return a


def unpack(params, channels):
    """Parameter vector -> list of (W[27][cin][cout], b[cout]) per layer."""
    out, off = [], 0
    for l in range(len(channels) - 1):
        ci, co = channels[l], channels[l + 1]
        W = np.asarray(params[off: off + 27 * ci * co], dtype=np.float64).reshape(27, ci, co)
        off += 27 * ci * co
        b = np.asarray(params[off: off + co], dtype=np.float64)
        off += co
        out.append((W, b))
    assert off == len(params)
    return out


def param_count(channels):
    return sum(27 * channels[l] * channels[l + 1] + channels[l + 1] for l in range(len(channels) - 1))


def conv(x, W, b):
    """One 3x3x3 periodic cross-correlation: x [cin][z][y][x] -> [cout][z][y][x]."""
    y = np.zeros((W.shape[2],) + x.shape[1:])
    for t in range(27):
        y += np.einsum("izyx,io->ozyx", shift(x, t), W[t])
    return y + b[:, None, None, None]


def forward(params, channels, xn, store=None):
    """Network output for a normalised input; also the list of layer inputs."""
    store = store or _same
    layers = unpack(params, channels)
    h, inputs = store(np.asarray(xn, dtype=np.float64)), []
    for l, (W, b) in enumerate(layers):
        inputs.append(h)
        pre = conv(h, store(W), b)
        h = pre if l == len(layers) - 1 else store(np.maximum(pre, 0.0))
    return h, inputs


def loss_and_grad(params, channels, x, target, mean, std, store=None, out_std=None, out_offset=0):
    """Loss of one sample and its gradient with respect to the parameters;
    output c is compared with field out_offset + c."""
    store = store or _same
    mean = np.asarray(mean, dtype=np.float64)[:, None, None, None]
    std = np.asarray(std, dtype=np.float64)[:, None, None, None]
    x = np.asarray(x, dtype=np.float64)
    C = channels[-1]
    y, inputs = forward(params, channels, (x - mean) / std, store)
    o = out_offset
    s = std[o:o + C] if out_std is None else np.asarray(out_std, dtype=np.float64)[:, None, None, None]
    r = y + (x[o:o + C] - np.asarray(target, dtype=np.float64)[o:o + C]) / s
    V = r[0].size
    loss = float((r ** 2).sum() / (C * V))
    d = store(2.0 * r / (C * V))  # dL/dy
    layers = unpack(params, channels)
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        h = inputs[l]
        dW = np.stack([np.einsum("izyx,ozyx->io", shift(h, t), d) for t in range(27)])
        db = d.sum(axis=(1, 2, 3))
        grads.append((dW, db))
        if l > 0:
            # dL/dh(v) = sum_t sum_o d[o](v - s_t) W[t][i][o], then the ReLU that produced h
            dh = np.zeros(h.shape)
            Ws = store(W)
            for t in range(27):
                dh += np.einsum("ozyx,io->izyx", shift(d, t, sign=-1), Ws[t])
            d = store(dh * (h > 0.0))
    g = []
    for dW, db in reversed(grads):
        g.append(dW.ravel())
        g.append(db)
    return loss, np.concatenate(g)


def adam_step(p, g, m, v, lr, b1, b2, eps, t):
    """One Adam update (in place), bias-corrected with step count t >= 1."""
    m[:] = b1 * m + (1.0 - b1) * g
    v[:] = b2 * v + (1.0 - b2) * g * g
    p -= lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps)
    return p


def box_filter(rho, u, T, factor, Cv):
    """Coarse moments: means of rho, rho u and rho E over factor^D blocks
    (D = number of velocity components; the z factor is 1 in 2-D)."""
    D = u.shape[0]
    fz = factor if D == 3 else 1

    def blocks(a):
        nz, ny, nx = a.shape
        return a.reshape(nz // fz, fz, ny // factor, factor, nx // factor, factor).mean(axis=(1, 3, 5))

    E = Cv * T + 0.5 * (u ** 2).sum(0)
    r = blocks(rho)
    uc = np.stack([blocks(rho * u[a]) / r for a in range(D)])
    Ec = blocks(rho * E) / r
    return r, uc, (Ec - 0.5 * (uc ** 2).sum(0)) / Cv


def kinetic_energy_spectrum(u):
    """E(k) of u [D][z][y][x] (or [D][1][y][x]) by integer shells k = round(|k|),
    E(k) = sum over the shell of |u_hat|^2 / 2 with u_hat = fft / N."""
    D = u.shape[0]
    axes = tuple(range(1, u.ndim))
    uh = np.fft.fftn(u, axes=axes) / u[0].size
    freqs = [np.fft.fftfreq(n, d=1.0 / n) for n in u.shape[1:]]
    K = np.meshgrid(*freqs, indexing="ij")
    kmag = np.sqrt(sum(k ** 2 for k in K))
    shell = np.rint(kmag).astype(np.int64)
    e = 0.5 * (np.abs(uh) ** 2).sum(0)
    return np.bincount(shell.ravel(), e.ravel())
