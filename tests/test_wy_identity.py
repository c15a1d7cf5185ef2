"""The compact-WY identity both T-factor kernels use (stage-1 panels, BT2 blocks).

For Householder reflectors H_j = I - tau_j v_j v_j^H with real tau_j, the
product H_0 H_1 ... H_{k-1} equals I - V T V^H with T upper triangular.  The
classic construction is the forward column recurrence
    T[j, j] = tau_j,  T[0:j, j] = -tau_j T[0:j, 0:j] (V^H V)[0:j, j];
the kernels instead solve T = U^{-1}, U = diag(1/tau) + (strict upper part of
V^H V), column by column by back substitution,
    T[i, c] = -tau_i sum_{k = i+1 .. c} G[i, k] T[k, c],
which needs no division by tau, so a zero tau (no reflector) just gives a
zero row and column.  These tests check, in plain numpy on the CPU, that the
two constructions agree and reproduce the reflector product, including the
zero-tau case.  They exercise no GPU code.
"""
import numpy as np


def _reflectors(rng, m, k, zero=()):
    """Unit lower-trapezoidal V (m x k) and real tau of genuine Householder
    reflectors (tau = 2 / |v|^2 makes each H_j unitary); columns in `zero`
    get tau = 0."""
    V = np.zeros((m, k), complex)
    tau = np.zeros(k)
    for j in range(k):
        v = rng.standard_normal(m) + 1j * rng.standard_normal(m)
        v[:j] = 0.0
        v[j] = 1.0
        V[:, j] = v
        tau[j] = 0.0 if j in zero else 2.0 / np.vdot(v, v).real
    return V, tau


def _t_forward(G, tau):
    k = len(tau)
    T = np.zeros((k, k), complex)
    for j in range(k):
        T[j, j] = tau[j]
        if j:
            T[:j, j] = -tau[j] * (T[:j, :j] @ G[:j, j])
    return T


def _t_backsub(G, tau):
    k = len(tau)
    T = np.zeros((k, k), complex)
    for c in range(k):
        T[c, c] = tau[c]
        for i in range(c - 1, -1, -1):
            T[i, c] = -tau[i] * (G[i, i + 1:c + 1] @ T[i + 1:c + 1, c])
    return T


def _product(V, tau):
    m = V.shape[0]
    Q = np.eye(m, dtype=complex)
    for j in range(V.shape[1]):
        v = V[:, j:j + 1]
        Q = Q @ (np.eye(m) - tau[j] * (v @ v.conj().T))
    return Q


def test_backsub_equals_forward_recurrence_and_product():
    rng = np.random.default_rng(7)
    for m, k in ((9, 4), (40, 16), (96, 32), (130, 64)):
        V, tau = _reflectors(rng, m, k)
        G = V.conj().T @ V
        Tf, Tb = _t_forward(G, tau), _t_backsub(G, tau)
        scale = np.abs(Tf).max()
        assert np.abs(Tb - Tf).max() <= 1e-12 * scale
        # the inverse form: U T = I with U = diag(1/tau) + striu(G)
        U = np.diag(1.0 / tau) + np.triu(G, 1)
        assert np.abs(U @ Tb - np.eye(k)).max() <= 1e-10
        Q = _product(V, tau)
        assert np.abs(np.eye(m) - V @ Tb @ V.conj().T - Q).max() <= 1e-12
        assert np.allclose(Tb, np.triu(Tb))


def test_zero_tau_gives_zero_row_and_column():
    rng = np.random.default_rng(11)
    m, k = 50, 12
    zero = (0, 5, 11)
    V, tau = _reflectors(rng, m, k, zero)
    G = V.conj().T @ V
    Tf, Tb = _t_forward(G, tau), _t_backsub(G, tau)
    assert np.abs(Tb - Tf).max() <= 1e-12 * np.abs(Tf).max()
    for j in zero:
        assert not Tb[j, :].any() and not Tb[:, j].any()
    Q = _product(V, tau)
    assert np.abs(np.eye(m) - V @ Tb @ V.conj().T - Q).max() <= 1e-12
