"""Oracle: TDSLDA time evolution of the quasiparticle wavefunctions (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Eq. (TDSLDA): i d/dt phi_j = H(t) phi_j for every evolved state
phi_j = [u_j; v_j], with the quasiparticle Hamiltonian
    H = [[h, Delta], [Delta^*, -h^*]],   h = -nabla^2/2 + U(r, t) - mu,
the kinetic term applied as F^-1 (k^2/2) F (numpy FFT along every lattice
axis, momenta k = 2 pi n / N as in "Numerical setup and implementation").  The
mean fields follow the densities of the evolved states ("each of which is
computed from the orbitals via a reduction"), with the zero-temperature
occupations of the time-dependent runs:
    n = 2 sum_j |v_j|^2,  nu = sum_j u_j v_j^*,
    U = Vext + B eps_F(n),  Delta = g nu   (complex: the phase evolves freely).
With self_consistent=False the fields stay those given at the start (a fixed
H), which the closed-form pins use.

Integrator ("Performance of the Time Evolution Algorithm": fifth-order
multistep Adams-Bashforth-Moulton predictor-corrector, two evaluations of H
per step), with f = -i H[phi] phi and f_k = f(phi_k):
    predictor  phi* = phi_k + dt/720 (1901 f_k - 2774 f_{k-1} + 2616 f_{k-2}
                                      - 1274 f_{k-3} + 251 f_{k-4})
    evaluate   f* = f(phi*)
    corrector  phi_{k+1} = phi_k + dt/720 (251 f* + 646 f_k - 264 f_{k-1}
                                           + 106 f_{k-2} - 19 f_{k-3})
    evaluate   f_{k+1} = f(phi_{k+1})
(the five-step Adams-Bashforth and four-step Adams-Moulton formulas, both of
order five).  The four steps that fill the history take the classical
fourth-order Runge-Kutta method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .scf import eps_F

AB5 = np.array([1901.0, -2774.0, 2616.0, -1274.0, 251.0]) / 720.0   # f_k, f_{k-1}, ..., f_{k-4}
AM5 = np.array([251.0, 646.0, -264.0, 106.0, -19.0]) / 720.0        # f*, f_k, f_{k-1}, f_{k-2}, f_{k-3}


@dataclass
class TdParams:
    B: float = 0.0
    g: float = 0.0
    self_consistent: bool = True


def kinetic(dims, psi: np.ndarray) -> np.ndarray:
    """-nabla^2/2 psi = F^-1 (k^2/2 F psi) for psi [nsites, m] (x fastest)."""
    dims = tuple(int(v) for v in dims)
    m = psi.shape[1]
    a = psi.reshape(tuple(reversed(dims)) + (m,))      # numpy axes (z, y, x, col)
    A = np.fft.fftn(a, axes=tuple(range(len(dims))))
    k2 = np.zeros(tuple(reversed(dims)))
    for ax, N in enumerate(dims):
        k = 2.0 * math.pi * np.fft.fftfreq(N) * 1.0      # 2 pi n / N, n = -N/2 .. N/2-1 (wrapped)
        k[N // 2] = -math.pi                              # Nyquist mode sits at n = -N/2
        shape = [1] * len(dims)
        shape[len(dims) - 1 - ax] = N
        k2 = k2 + (k * k).reshape(shape)
    A *= (0.5 * k2)[..., None]
    return np.fft.ifftn(A, axes=tuple(range(len(dims)))).reshape(psi.shape)


def densities(Phi: np.ndarray, nsites: int):
    u, v = Phi[:nsites], Phi[nsites:]
    return 2.0 * np.sum(np.abs(v) ** 2, axis=1), np.sum(u * v.conj(), axis=1)


def fields(dims, Vext, Phi, p: TdParams, U0=None, D0=None):
    """Mean fields (U, Delta) of the state Phi (or the frozen U0, D0)."""
    if not p.self_consistent:
        return U0, D0
    n, nu = densities(Phi, int(np.prod(dims)))
    return Vext + p.B * eps_F(n, len(dims)), p.g * nu


def apply_h(dims, U, Delta, mu, Phi) -> np.ndarray:
    """H Phi for the BdG Hamiltonian with the local fields U (real), Delta (complex)."""
    ns = int(np.prod(dims))
    u, v = Phi[:ns], Phi[ns:]
    Tu, Tv = kinetic(dims, u), kinetic(dims, v)
    loc = (U - mu)[:, None]
    top = Tu + loc * u + Delta[:, None] * v
    bot = Delta.conj()[:, None] * u - (Tv + loc * v)   # -h^* v with h real
    return np.vstack([top, bot])


def rhs(dims, Vext, mu, p, Phi, U0=None, D0=None):
    U, D = fields(dims, Vext, Phi, p, U0, D0)
    return -1j * apply_h(dims, U, D, mu, Phi)


def evolve(dims, Vext, mu, p: TdParams, Phi0: np.ndarray, dt: float, nsteps: int, U0=None, D0=None):
    """Phi after nsteps steps of size dt (ABM5 after four RK4 steps)."""
    f = lambda Phi: rhs(dims, Vext, mu, p, Phi, U0, D0)  # noqa: E731
    Phi = np.array(Phi0, dtype=np.complex128, copy=True)
    hist = [f(Phi)]                       # hist[0] = f_k, hist[1] = f_{k-1}, ...
    for step in range(nsteps):
        if step < 4:
            k1 = hist[0]
            k2 = f(Phi + 0.5 * dt * k1)
            k3 = f(Phi + 0.5 * dt * k2)
            k4 = f(Phi + dt * k3)
            Phi = Phi + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        else:
            pred = Phi + dt * sum(c * fk for c, fk in zip(AB5, hist[:5]))
            fp = f(pred)
            Phi = Phi + dt * (AM5[0] * fp + sum(c * fk for c, fk in zip(AM5[1:], hist[:4])))
        hist.insert(0, f(Phi))
        del hist[5:]
    return Phi
