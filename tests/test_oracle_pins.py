"""Pins for the oracle's helpers that serve the large-size parity tests and
the network's optimiser.

* ``assemble_entries`` (entries of H one by one) equals the dense ``assemble``
  entry for entry;
* ``apply_h`` (H applied axis by axis, no dense H) equals ``assemble(...) @ z``
  and, for uniform fields, reproduces the closed form of a plane wave:
  the spectral kinetic operator of "Numerical setup and implementation"
  multiplies e^{i k r} by k^2/2, so for constant U and Delta the 2x2 block
  [[eps_k + U - mu, Delta], [conj(Delta), -(eps_k + U - mu)]] acts on the
  amplitudes (a, b) of [a e^{ikr}; b e^{ikr}];
* ``oracle.net.adam_step`` reproduces two steps of Kingma & Ba's Algorithm 1
  computed by hand (bias corrections 1 - beta^t, epsilon added to the square
  root of the corrected second moment), with beta2 and epsilon chosen so that
  a missing bias correction or epsilon moved inside the root changes the
  result in the third digit.
"""
import itertools

import numpy as np
import pytest

from paper_2310_03341_amd import inputs


def _vortex_workload(dims, seed):
    ns = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    D = 0.3 * np.exp(1j * rng.uniform(-np.pi, np.pi, ns)) * rng.uniform(0.2, 1.0, ns)
    return inputs.Workload("pin", tuple(dims), rng.uniform(-0.5, 0.5, ns), D, 0.7)


@pytest.mark.parametrize("dims", [(4, 4, 2), (6, 6, 4), (8, 6)])
def test_assemble_entries_equals_assemble(orc, dims):
    w = _vortex_workload(dims, 11)
    H = orc.assemble_workload(w)
    n = H.shape[0]
    rows, cols = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    got = orc.assemble_entries(w.dims, w.U, w.Delta, w.mu, rows.ravel(), cols.ravel())
    assert np.abs(got - H[rows.ravel(), cols.ravel()]).max() == 0.0


@pytest.mark.parametrize("dims", [(8,), (6, 4), (4, 4, 2), (6, 4, 4)])
def test_apply_h_equals_dense_product(orc, dims):
    w = _vortex_workload(dims, 12)
    H = orc.assemble_workload(w)
    rng = np.random.default_rng(3)
    Z = rng.standard_normal((H.shape[0], 7)) + 1j * rng.standard_normal((H.shape[0], 7))
    got = orc.apply_h(w.dims, w.U, w.Delta, w.mu, Z)
    assert np.abs(got - H @ Z).max() < 1e-13 * np.abs(H @ Z).max()
    # a single vector gives a vector (BLAS may sum in another order)
    one = orc.apply_h(w.dims, w.U, w.Delta, w.mu, Z[:, 2])
    assert one.shape == (H.shape[0],)
    assert np.abs(one - got[:, 2]).max() < 1e-14 * np.abs(got).max()


@pytest.mark.parametrize("dims", [(8,), (6, 4), (4, 6, 2)])
def test_apply_h_plane_waves_closed_form(orc, dims):
    U0, D0, mu = 0.15, 0.2 - 0.35j, 0.9
    w = inputs.uniform(dims, U0, D0, mu)
    ns = w.nsites
    xs = inputs.coords(dims)
    for ms in itertools.product(*[(-N // 2, -1, 0, 1, N // 2 - 1) for N in dims]):
        k = [2 * np.pi * mm / N for mm, N in zip(ms, dims)]
        phase = np.exp(1j * sum(kk * x for kk, x in zip(k, xs)))
        eps = sum(kk * kk / 2 for kk in k)
        a, b = 0.6 + 0.1j, -0.3 + 0.7j
        z = np.concatenate([a * phase, b * phase])
        got = orc.apply_h(dims, w.U, w.Delta, mu, z)
        xi = eps + U0 - mu
        ref = np.concatenate([(xi * a + D0 * b) * phase, (np.conj(D0) * a - xi * b) * phase])
        assert np.abs(got - ref).max() < 1e-12, ms


def test_adam_two_steps_by_hand():
    from oracle import net
    # lr 0.1, beta1 0.9, beta2 0.99, eps 0.01; p0 = (1, -2)
    # step 1, g = (0.5, 2): m = (0.05, 0.2), v = (0.0025, 0.04),
    #   m^ = m / 0.1 = (0.5, 2), v^ = v / 0.01 = (0.25, 4), sqrt v^ = (0.5, 2),
    #   p1 = p0 - 0.1 m^ / (sqrt v^ + 0.01) = (1 - 0.05/0.51, -2 - 0.2/2.01)
    # step 2, g = (-1, 1): m = 0.9 m + 0.1 g = (-0.055, 0.28),
    #   v = 0.99 v + 0.01 g^2 = (0.012475, 0.0496),
    #   m^ = m / 0.19, v^ = v / 0.0199, p2 = p1 - 0.1 m^ / (sqrt v^ + 0.01)
    p1_ref = np.array([0.901960784313725490196, -2.099502487562189054726])
    p2_ref = np.array([0.938065549408075298566, -2.192259752883973728889])
    m_ref = np.array([-0.055, 0.28])
    v_ref = np.array([0.012475, 0.0496])
    p = [np.array([1.0, -2.0])]
    m, v = [np.zeros(2)], [np.zeros(2)]
    p = net.adam_step(p, [np.array([0.5, 2.0])], m, v, 1, lr=0.1, b1=0.9, b2=0.99, eps=0.01)
    assert np.abs(p[0] - p1_ref).max() < 1e-15
    p = net.adam_step(p, [np.array([-1.0, 1.0])], m, v, 2, lr=0.1, b1=0.9, b2=0.99, eps=0.01)
    assert np.abs(m[0] - m_ref).max() < 1e-15 and np.abs(v[0] - v_ref).max() < 1e-15
    assert np.abs(p[0] - p2_ref).max() < 1e-15
