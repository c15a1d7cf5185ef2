"""Pins for the TDSLDA evolution oracle: the integrator's formulas on
polynomials, the spectral kinetic term, exact phases of eigenstates of a fixed
H, the free-particle propagator, unitarity, and the stationarity of a
self-consistent uniform state."""
import math

import numpy as np
import pytest

import oracle
from oracle import scf
from oracle import tdslda as td
from paper_2310_03341_amd import inputs


def test_abm_formulas_integrate_quartics_exactly():
    """Both five-step formulas are exact for y' = t^k, k <= 4 (order five), and
    not for k = 5; a wrong coefficient breaks one of these."""
    h = 0.1
    for k in range(6):
        ts = np.array([0.0, -h, -2 * h, -3 * h, -4 * h])  # t_k, t_{k-1}, ...
        f = ts ** k
        exact = h ** (k + 1) / (k + 1)                     # int_0^h t^k dt
        ab = h * np.dot(td.AB5, f)
        am = h * (td.AM5[0] * h ** k + np.dot(td.AM5[1:], f[:4]))
        if k <= 4:
            assert abs(ab - exact) < 1e-15 and abs(am - exact) < 1e-15, k
        else:
            assert abs(ab - exact) > 1e-9 and abs(am - exact) > 1e-11
    assert abs(td.AB5.sum() - 1.0) < 1e-15 and abs(td.AM5.sum() - 1.0) < 1e-15


def test_kinetic_matches_direct_fourier_sum():
    """FFT kinetic term against the direct-sum kinetic matrices of the assembly
    oracle (Kronecker sum over the axes), and plane waves as eigenvectors."""
    rng = np.random.default_rng(1)
    for dims in ((8,), (6, 4), (4, 6, 4)):
        ns = int(np.prod(dims))
        psi = rng.standard_normal((ns, 3)) + 1j * rng.standard_normal((ns, 3))
        T = np.zeros((ns, ns))
        stride = 1
        for N in dims:
            t1 = oracle.kinetic_1d(N)
            T += np.kron(np.kron(np.eye(ns // (stride * N)), t1), np.eye(stride))
            stride *= N
        assert np.abs(td.kinetic(dims, psi) - T @ psi).max() < 1e-12
    N = 8
    x = np.arange(N)
    for n in range(-N // 2, N // 2):
        k = 2 * math.pi * n / N
        pw = np.exp(1j * k * x)[:, None]
        assert np.abs(td.kinetic((N,), pw) - 0.5 * k * k * pw).max() < 1e-13


def test_eigenstates_of_a_fixed_h_pick_up_exact_phases(orc):
    """With the fields frozen, an eigenvector of H with energy E evolves as
    e^{-iEt}; the fifth-order integrator stays within its error bound."""
    w = inputs.uniform((6, 4), 0.1, 0.3 + 0.1j, 1.0)
    H = orc.assemble_workload(w)
    W, Z = orc.eigh(H)
    idx = [0, 5, 20, 47]
    Phi0 = Z[:, idx]
    dt, steps = 0.01, 200
    t = dt * steps
    p = td.TdParams(self_consistent=False)
    Phi = td.evolve(w.dims, np.zeros(w.nsites), w.mu, p, Phi0, dt, steps,
                    U0=np.full(w.nsites, 0.1), D0=np.full(w.nsites, 0.3 + 0.1j))
    exact = Phi0 * np.exp(-1j * W[idx] * t)
    # for y' = -iEy the fifth-order corrector leaves a global error of about
    # |C| (dt E)^5 |E| t with C = -3/160, its error constant (factor 2 margin)
    bound = 2 * (3 / 160) * (dt * np.abs(W[idx])) ** 5 * np.abs(W[idx]) * t + 1e-13
    err = np.abs(Phi - exact).max(axis=0)
    assert np.all(err < bound), (err, bound)
    # and a step twice as long is worse by about 2^5
    Phi2 = td.evolve(w.dims, np.zeros(w.nsites), w.mu, p, Phi0, 2 * dt, steps // 2,
                     U0=np.full(w.nsites, 0.1), D0=np.full(w.nsites, 0.3 + 0.1j))
    e1, e2 = np.abs(Phi - exact).max(), np.abs(Phi2 - exact).max()
    assert 16 < e2 / e1 < 64, (e1, e2)


def test_free_particle_propagator():
    """No fields, no pairing: u(t) = F^-1 e^{-i (k^2/2 - mu) t} F u(0)."""
    dims = (16,)
    ns = 16
    x = np.arange(ns)
    u0 = np.exp(-0.5 * ((x - 8.0) / 2.0) ** 2) * np.exp(0.7j * x)
    u0 /= np.linalg.norm(u0)
    Phi0 = np.concatenate([u0, np.zeros(ns)])[:, None]
    mu, dt, steps = 0.2, 0.005, 400
    p = td.TdParams(self_consistent=False)
    Phi = td.evolve(dims, np.zeros(ns), mu, p, Phi0, dt, steps, U0=np.zeros(ns), D0=np.zeros(ns, complex))
    k = 2 * math.pi * np.fft.fftfreq(ns)
    exact = np.fft.ifft(np.exp(-1j * (0.5 * k * k - mu) * dt * steps) * np.fft.fft(u0))
    assert np.abs(Phi[:ns, 0] - exact).max() < 1e-9
    assert np.abs(Phi[ns:]).max() == 0.0


def test_self_consistent_evolution_is_unitary_and_uniform_state_stationary(orc):
    """Uniform gas at its gap-equation fixed point (B = 0): a stationary state
    of eq. (TDSLDA), so the densities stay put; and any evolution keeps the
    states orthonormal (the Hamiltonian is Hermitian at every instant)."""
    dims = (8, 8)
    mu, g = 1.0, inputs.ScfParams().g
    ns = 64
    d = 0.3
    for _ in range(300):  # gap equation Delta = g nu, uniform
        _, nu = scf.uniform_densities(dims, 0.0, d, mu, math.pi ** 2 / 2)
        d = g * abs(nu)
    w = inputs.uniform(dims, 0.0, d, mu)
    H = orc.assemble_workload(w)
    W, Z = orc.eigh(H, np.nextafter(0.0, 1.0), math.pi ** 2 / 2)
    p = td.TdParams(B=0.0, g=g)
    n0, nu0 = td.densities(Z, ns)
    # dt = 0.004: about the paper's 286 steps per unit time
    Phi = td.evolve(dims, np.zeros(ns), mu, p, Z, 0.004, 250)
    n1, nu1 = td.densities(Phi, ns)
    assert np.abs(n1 - n0).max() < 1e-9 and np.abs(nu1 - nu0).max() < 1e-9
    # a perturbed start moves but stays orthonormal to O(dt^5)
    rng = np.random.default_rng(3)
    Vext = 0.2 * rng.standard_normal(ns)
    p2 = td.TdParams(B=-0.3, g=g)
    Phi = td.evolve(dims, Vext, mu, p2, Z, 0.004, 250)
    n2, _ = td.densities(Phi, ns)
    assert np.abs(n2 - n0).max() > 1e-3
    assert np.abs(Phi.conj().T @ Phi - np.eye(Z.shape[1])).max() < 1e-9
