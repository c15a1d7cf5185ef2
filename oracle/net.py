"""Oracle: the start-field network of the learned SCF start (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A plain definition of what the GPU kernels compute (the learned extension of
the hot path; the paper starts its SLDA iterations from coarser lattices
instead, "Performance of the Matrix Diagonalization Algorithm"):

  x0 = (Vext - mu, cos theta, sin theta)           3 channels on the periodic lattice
  x1 = relu(conv(x0; W1, b1))                      C channels
  x2 = relu(conv(x1; W2, b2))
  x3 = relu(conv(x2; W3, b3))
  y  = conv(x3; W4, b4)                            2 channels: U - Vext, |Delta|
  conv(x; W, b)[o, p] = b[o] + sum_{c, dy, dx} W[o, c, dy, dx] x[c, p + (dy-1, dx-1)]  (periodic)
  loss = mean over batch, channels and sites of (y - target)^2

Layout: arrays are (batch, channel, Ny, Nx) with x fastest, matching the
lattice site order r = x + Nx y.  Backward is written out by hand from these
definitions (no autograd); Adam follows Kingma & Ba (2015).
"""
from __future__ import annotations

import numpy as np


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Periodic 3x3 convolution (cross-correlation) with bias."""
    B, C, Ny, Nx = x.shape
    O = W.shape[0]
    y = np.zeros((B, O, Ny, Nx))
    for dy in range(3):
        for dx in range(3):
            xs = np.roll(x, shift=(-(dy - 1), -(dx - 1)), axis=(2, 3))  # xs[p] = x[p + d]
            y += np.einsum("oc,bcyx->boyx", W[:, :, dy, dx], xs)
    return y + b[None, :, None, None]


def conv_backward(x, W, gy):
    """Gradients of conv w.r.t. x, W and b given the output gradient gy."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for dy in range(3):
        for dx in range(3):
            xs = np.roll(x, shift=(-(dy - 1), -(dx - 1)), axis=(2, 3))
            gW[:, :, dy, dx] = np.einsum("boyx,bcyx->oc", gy, xs)
            t = np.einsum("oc,boyx->bcyx", W[:, :, dy, dx], gy)
            gx += np.roll(t, shift=(dy - 1, dx - 1), axis=(2, 3))
    gb = gy.sum(axis=(0, 2, 3))
    return gx, gW, gb


def init_params(C: int, seed: int = 0):
    """He-style initialisation; returns [W1, b1, ..., W4, b4]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(C, 3), (C, C), (C, C), (2, C)]
    params = []
    for (o, c) in shapes:
        W = rng.standard_normal((o, c, 3, 3)) * np.sqrt(2.0 / (9 * c))
        params += [W, np.zeros(o)]
    params[-2] *= 0.1
    return params


def forward(params, x0):
    acts = [x0]
    h = x0
    for layer in range(4):
        W, b = params[2 * layer], params[2 * layer + 1]
        z = conv(h, W, b)
        h = np.maximum(z, 0.0) if layer < 3 else z
        acts.append(h)
    return h, acts


def loss_and_grads(params, x0, target):
    y, acts = forward(params, x0)
    diff = y - target
    loss = np.mean(diff ** 2)
    g = 2.0 * diff / diff.size
    grads = [None] * 8
    for layer in range(3, -1, -1):
        W = params[2 * layer]
        if layer < 3:
            g = g * (acts[layer + 1] > 0.0)
        gx, gW, gb = conv_backward(acts[layer], W, g)
        grads[2 * layer], grads[2 * layer + 1] = gW, gb
        g = gx
    return loss, grads


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    out = []
    for i, (p, g) in enumerate(zip(params, grads)):
        m[i] = b1 * m[i] + (1 - b1) * g
        v[i] = b2 * v[i] + (1 - b2) * g * g
        mh = m[i] / (1 - b1 ** t)
        vh = v[i] / (1 - b2 ** t)
        out.append(p - lr * mh / (np.sqrt(vh) + eps))
    return out


def features(Vext, theta, mu, dims):
    """Input channels (Vext - mu, cos theta, sin theta) shaped (3, Ny, Nx)."""
    Nx, Ny = dims
    f = np.stack([Vext - mu, np.cos(theta), np.sin(theta)])
    return f.reshape(3, Ny, Nx)
