"""Oracle: one step of the static SLDA self-consistency (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the paper's "Methods": quasiparticle states of eq. (stHpsi) with
0 < E_n < E_c (E_c = pi^2/2) and the densities of eq. (densities2) with the
Fermi function f_T(E) = 1 / (1 + exp(E/T)):
    n(r)  = 2 sum_n (|v_n(r)|^2 f_T(-E_n) + |u_n(r)|^2 f_T(E_n)),
    nu(r) = sum_n u_n(r) v_n(r)^* (f_T(-E_n) - f_T(E_n)),
which at T = 0 become n = 2 sum |v_n|^2 and nu = sum u_n v_n^*;
mean fields with A = 1 (no current term, h = -nabla^2/2 + U - mu) and the
pairing field Delta = g nu with its phase held fixed ("Initial state
preparation": only |Delta| is iterated).  The density dependence of U is a
synthetic functional U = Vext + B eps_F(n) (the paper's A, B, C constants are
not printed); linear mixing closes the step.

Cut-off regularisation ("Density functional theory for superfluid fermions",
the Lambda_c expression): with the energy cut-off E_c the anomalous density
diverges with the cut-off momentum, and the functional fixes the finite
combination 1/g_c + Lambda_c instead of g_c.  Here g (positive = attractive,
Delta = g nu) plays the finite coupling g0, and the step uses the local
    g_eff(r) = 1 / (1/g0 + Lambda_c(r)),
    Lambda_c = (1 / 2 pi^2) (k_c - (k_0/2) ln((k_c + k_0)/(k_c - k_0)))
(hbar = m = 1), the principal-value integral of 1/(k^2 - k_0^2) over the
momentum ball |k| < k_c, with the local momenta k_c^2/2 = E_c + mu - U(r)
and k_0^2/2 = mu - U(r) (k_0 ~ k_F).  Where mu < U(r) the same integral has
no pole: (k_c - kappa atan(k_c/kappa)) / 2 pi^2 with kappa^2 = -k_0^2.  The
paper gives the three-dimensional form only, so regularisation is defined on
3-D lattices.

Multigrid start ("Performance of the Matrix Diagonalization Algorithm": the
solution on a coarser lattice starts the next finer one).  Lengths are in
lattice spacings on every level, so the coarse level with spacing s fine
spacings is the same physical problem in rescaled units: fields sampled at
every s-th fine site (injection), energies times s^2 (Vext, mu, U, |Delta|,
E_c keeps pi^2/2 of its own lattice), densities times s^d and couplings
g times s^(2-d).  ``fourier_interp`` carries the converged coarse fields back
as the trigonometric interpolant of the coarse samples (Nyquist coefficient
split evenly between +-N/2 so that a real field stays real).
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


def fermi(E, T: float):
    """f_T(E) = 1 / (1 + exp(E/T)) of eq. (densities2); T = 0: 1 for E < 0,
    0 for E > 0 (1/2 at E = 0)."""
    E = np.asarray(E, dtype=np.float64)
    if T == 0.0:
        return np.where(E < 0, 1.0, np.where(E > 0, 0.0, 0.5))
    x = E / T
    # 1 / (1 + e^x) written so that neither branch overflows
    return np.where(x > 0, np.exp(-np.abs(x)) / (1.0 + np.exp(-np.abs(x))), 1.0 / (1.0 + np.exp(-np.abs(x))))


def densities(W: np.ndarray, Z: np.ndarray, nsites: int, T: float = 0.0):
    """n(r), nu(r) of eq. (densities2) from eigenpairs (already restricted to
    0 < E < Ec)."""
    u, v = Z[:nsites], Z[nsites:]
    fp, fm = fermi(-W, T), fermi(W, T)
    n = 2.0 * (np.abs(v) ** 2 @ fp + np.abs(u) ** 2 @ fm)
    nu = (u * v.conj()) @ (fp - fm)
    return n, nu


def lambda_c(kc2, k02):
    """Lambda_c of the cut-off regularisation (3-D, hbar = m = 1) from the local
    k_c^2 and k_0^2: (1/2 pi^2) PV int_0^k_c k^2 dk / (k^2 - k_0^2); zero where
    k_c^2 <= 0 (no state below the cut-off)."""
    kc2 = np.asarray(kc2, dtype=np.float64)
    k02 = np.asarray(k02, dtype=np.float64)
    out = np.zeros(np.broadcast(kc2, k02).shape)
    kc2b, k02b = np.broadcast_arrays(kc2, k02)
    for i in np.ndindex(out.shape):
        a, b = float(kc2b[i]), float(k02b[i])
        if a <= 0.0:
            continue
        kc = math.sqrt(a)
        if b > 0.0:
            k0 = math.sqrt(b)
            val = kc - 0.5 * k0 * math.log((kc + k0) / (kc - k0))
        elif b < 0.0:
            ka = math.sqrt(-b)
            val = kc - ka * math.atan(kc / ka)
        else:
            val = kc
        out[i] = val / (2.0 * math.pi ** 2)
    return out


def g_effective(p, U, mu, ndim: int):
    """Coupling of the step: g, or 1/(1/g + Lambda_c(r)) with regularisation."""
    if not getattr(p, "regularize", 0):
        return np.full(np.shape(U), p.g)
    if ndim != 3:
        raise ValueError("the cut-off regularisation is defined for 3-D lattices")
    lam = lambda_c(2.0 * (p.Ec + mu - U), 2.0 * (mu - U))
    return 1.0 / (1.0 / p.g + lam)


def scf_step(dims, Vext, theta, mu, U, absDelta, p):
    """One SCF step; returns dict(U, absDelta, n, nu_abs, change, m)."""
    dims = tuple(int(v) for v in dims)
    ns = int(np.prod(dims))
    T = float(getattr(p, "T", 0.0))
    Delta = absDelta * np.exp(1j * theta)
    H = assemble(dims, U, Delta, mu)
    W, Z = eigh(H, np.nextafter(0.0, 1.0), p.Ec)
    n, nu = densities(W, Z, ns, T)
    U_new = Vext + p.B * eps_F(n, len(dims))
    D_new = g_effective(p, U, mu, len(dims)) * np.abs(nu)
    change = max(np.abs(U_new - U).max(), np.abs(D_new - absDelta).max())
    return {
        "U": (1.0 - p.alpha) * U + p.alpha * U_new,
        "absDelta": (1.0 - p.alpha) * absDelta + p.alpha * D_new,
        "n": n,
        "nu_abs": np.abs(nu),
        "change": change,
        "m": W.size,
    }


def uniform_densities(dims, U0, delta0, mu, Ec, T: float = 0.0):
    """Closed form for uniform fields: plane-wave quasiparticles (u_k, v_k) with
    |u|^2, |v|^2 = (1 +- xi/E)/2 and u v^* = Delta/2E give, with
    f_T(-E) - f_T(E) = tanh(E/2T) and f_T(-E) + f_T(E) = 1,
    n = N^-d sum_k (1 - (xi_k/E_k) tanh(E_k/2T)),
    nu = N^-d sum_k (Delta/2E_k) tanh(E_k/2T)   over 0 < E_k < Ec
    (tanh = 1 at T = 0)."""
    eps = np.zeros(())
    for N in dims:
        k = 2.0 * math.pi * np.arange(-N // 2, N // 2) / N
        eps = np.add.outer(eps, k * k / 2.0)
    xi = eps.ravel() + U0 - mu
    E = np.sqrt(xi ** 2 + abs(delta0) ** 2)
    sel = (E > 0) & (E < Ec)
    N = int(np.prod(dims))
    th = np.ones(np.count_nonzero(sel)) if T == 0.0 else np.tanh(E[sel] / (2.0 * T))
    n = np.sum(1.0 - xi[sel] / E[sel] * th) / N
    nu = np.sum(delta0 / (2.0 * E[sel]) * th) / N
    return n, nu


def fourier_interp_1d(N_c: int, N_f: int) -> np.ndarray:
    """N_f x N_c matrix of trigonometric interpolation: row x_f evaluates the
    interpolant of N_c periodic samples at x_f N_c / N_f (coarse units), the
    coefficient of the mode -N_c/2 split evenly between -N_c/2 and +N_c/2.
    Built as inverse FFT of zero-padded FFT columns."""
    P = np.zeros((N_f, N_c))
    for j in range(N_c):
        e = np.zeros(N_c)
        e[j] = 1.0
        c = np.fft.fft(e) / N_c                     # c[n], n = 0..N_c-1 (negative n wrapped)
        C = np.zeros(N_f, dtype=np.complex128)
        h = N_c // 2
        C[:h] = c[:h]                              # n = 0 .. h-1
        C[N_f - h + 1:] = c[h + 1:]                # n = -h+1 .. -1
        if N_c % 2 == 0:                           # Nyquist: half to -h, half to +h
            C[h] += 0.5 * c[h]
            C[N_f - h] += 0.5 * c[h]
        else:
            C[N_f - h] = c[h]
        P[:, j] = np.real(np.fft.ifft(C) * N_f)
    return P


def fourier_interp(dims_c, f, dims_f, scale: float = 1.0) -> np.ndarray:
    """scale x trigonometric interpolation of the periodic field f (x fastest)
    from the lattice dims_c to dims_f (each fine size >= the coarse one)."""
    g = np.asarray(f, dtype=np.float64).reshape(tuple(reversed(dims_c)))
    for ax, (Nc, Nf) in enumerate(zip(dims_c, dims_f)):
        P = fourier_interp_1d(Nc, Nf)
        axis = len(dims_c) - 1 - ax                # numpy axis of lattice axis ax
        g = np.moveaxis(np.tensordot(P, g, axes=([1], [axis])), 0, axis)
    return scale * g.ravel()


def restrict(dims_f, f, s: int, scale: float = 1.0) -> np.ndarray:
    """scale x f sampled at every s-th site of each axis (injection)."""
    g = np.asarray(f).reshape(tuple(reversed(dims_f)))
    sl = tuple(slice(0, None, s) for _ in dims_f)
    return scale * np.ascontiguousarray(g[sl]).ravel()
