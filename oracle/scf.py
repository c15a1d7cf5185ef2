"""Oracle: one step of the static SLDA self-consistency (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the paper's "Methods": quasiparticle states of eq. (stHpsi) with
0 < E_n < E_c (E_c = pi^2/2), zero-temperature occupations f_T(-E) = 1,
f_T(E) = 0 in eq. (densities2):
    n(r)  = 2 sum_n |v_n(r)|^2,     nu(r) = sum_n u_n(r) v_n(r)^*,
mean fields with A = 1 (no current term, h = -nabla^2/2 + U - mu) and the
pairing field Delta = g nu with its phase held fixed ("Initial state
preparation": only |Delta| is iterated).  The density dependence of U is a
synthetic functional U = Vext + B eps_F(n) (the paper's A, B, C constants are
not printed); linear mixing closes the step.
"""
from __future__ import annotations

import math

import numpy as np

from . import assemble, eigh


def eps_F(n: np.ndarray, ndim: int) -> np.ndarray:
    """Fermi energy of the two-species free gas at density n (hbar = m = 1)."""
    n = np.maximum(n, 0.0)
    if ndim == 2:
        return math.pi * n                         # n = kF^2 / (2 pi)
    if ndim == 3:
        return 0.5 * (3.0 * math.pi ** 2 * n) ** (2.0 / 3.0)   # n = kF^3 / (3 pi^2)
    return 0.5 * (math.pi * n / 2.0) ** 2          # 1D: n = 2 kF / pi


def densities(W: np.ndarray, Z: np.ndarray, nsites: int):
    """n(r), nu(r) from eigenpairs (already restricted to 0 < E < Ec)."""
    u, v = Z[:nsites], Z[nsites:]
    n = 2.0 * np.sum(np.abs(v) ** 2, axis=1)
    nu = np.sum(u * v.conj(), axis=1)
    return n, nu


def scf_step(dims, Vext, theta, mu, U, absDelta, p):
    """One SCF step; returns dict(U, absDelta, n, nu_abs, change, m)."""
    dims = tuple(int(v) for v in dims)
    ns = int(np.prod(dims))
    Delta = absDelta * np.exp(1j * theta)
    H = assemble(dims, U, Delta, mu)
    W, Z = eigh(H, np.nextafter(0.0, 1.0), p.Ec)
    n, nu = densities(W, Z, ns)
    U_new = Vext + p.B * eps_F(n, len(dims))
    D_new = p.g * np.abs(nu)
    change = max(np.abs(U_new - U).max(), np.abs(D_new - absDelta).max())
    return {
        "U": (1.0 - p.alpha) * U + p.alpha * U_new,
        "absDelta": (1.0 - p.alpha) * absDelta + p.alpha * D_new,
        "n": n,
        "nu_abs": np.abs(nu),
        "change": change,
        "m": W.size,
    }


def uniform_densities(dims, U0, delta0, mu, Ec):
    """Closed form for uniform fields: plane-wave quasiparticles give
    n = N^-d sum_k (1 - xi_k/E_k), nu = N^-d sum_k Delta/(2 E_k) over 0 < E_k < Ec."""
    eps = np.zeros(())
    for N in dims:
        k = 2.0 * math.pi * np.arange(-N // 2, N // 2) / N
        eps = np.add.outer(eps, k * k / 2.0)
    xi = eps.ravel() + U0 - mu
    E = np.sqrt(xi ** 2 + abs(delta0) ** 2)
    sel = (E > 0) & (E < Ec)
    N = int(np.prod(dims))
    n = np.sum(1.0 - xi[sel] / E[sel]) / N
    nu = np.sum(delta0 / (2.0 * E[sel])) / N
    return n, nu
