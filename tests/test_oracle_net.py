"""Pins for the start-field network oracle: brute-force convolution, finite
differences of the hand-written backward pass, Adam on a quadratic."""
import numpy as np

from oracle import net


def test_conv_matches_brute_force():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 5, 6))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = net.conv(x, W, b)
    B, C, Ny, Nx = x.shape
    ref = np.zeros((B, 4, Ny, Nx))
    for bb in range(B):
        for o in range(4):
            for yy in range(Ny):
                for xx in range(Nx):
                    s = b[o]
                    for c in range(C):
                        for dy in range(3):
                            for dx in range(3):
                                s += W[o, c, dy, dx] * x[bb, c, (yy + dy - 1) % Ny, (xx + dx - 1) % Nx]
                    ref[bb, o, yy, xx] = s
    assert np.abs(y - ref).max() < 1e-12


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    params = net.init_params(4, seed=3)
    x0 = rng.standard_normal((2, 3, 6, 6))
    target = rng.standard_normal((2, 2, 6, 6))
    loss, grads = net.loss_and_grads(params, x0, target)
    h = 1e-6
    for i, p in enumerate(params):
        idx = tuple(rng.integers(0, s) for s in p.shape)
        pp = [q.copy() for q in params]
        pp[i][idx] += h
        lp, _ = net.loss_and_grads(pp, x0, target)
        pp[i][idx] -= 2 * h
        lm, _ = net.loss_and_grads(pp, x0, target)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grads[i][idx]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, grads[i][idx])


def test_adam_minimises_quadratic():
    p = [np.array([3.0, -2.0])]
    m, v = [np.zeros(2)], [np.zeros(2)]
    for t in range(1, 3001):
        p = net.adam_step(p, [2 * p[0]], m, v, t, lr=1e-2)
    assert np.abs(p[0]).max() < 1e-3
