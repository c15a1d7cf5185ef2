"""Seeded synthetic inputs for the BdG eigenproblem workloads.

This module only draws fields (potential U(r), pairing field Delta(r), trap
potentials, vortex phases) from a seeded ``numpy.random.Generator``.  It holds
none of the method's arithmetic (no Hamiltonian, no eigen-solve, no density):
both the HIP path and the CPU oracle consume these arrays.

Conventions (paper, "Numerical setup and implementation"): periodic lattice,
spacing 1, site index r = x + Nx*(y + Ny*z) (x fastest).  Fields are returned
as flat float64 / complex128 arrays of length Nx*Ny*Nz.

Readings of the workload description that the paper leaves open:
  * U(r) is a sum of G Gaussians with centres uniform in the box, widths
    sigma ~ U(1.5, 4) in 2D and U(2, 6) in 3D, amplitudes ~ U(-0.5, 0.5),
    minimum-image periodic distance.
  * The pairing noise is 1e-3 * (xi1 + i xi2), xi ~ N(0, 1) per site.
  * Vortex geometry: 2D vortex centred on the site (N/2, N/2); 3D straight
    line along z through (Nx/2, Ny/2); ring of radius R in the plane z = Nz/2
    centred in the box, with healing length 3 and phase atan2(z - zc, rho - R).
  * Draw order: centres, widths, amplitudes, then noise.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One BdG matrix instance: lattice, fields and chemical potential."""

    name: str
    dims: Tuple[int, ...]
    U: np.ndarray          # float64, length prod(dims)
    Delta: np.ndarray      # complex128, length prod(dims)
    mu: float

    @property
    def nsites(self) -> int:
        return int(np.prod(self.dims))

    @property
    def n(self) -> int:
        return 2 * self.nsites


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def coords(dims: Sequence[int]):
    """Integer lattice coordinates, each flattened with x fastest."""
    grids = np.meshgrid(*[np.arange(d, dtype=np.float64) for d in dims],
                        indexing="ij")
    # meshgrid(ij) gives arrays shaped (Nx, Ny, Nz); Fortran flattening puts x fastest
    return [g.ravel(order="F") for g in grids]


def _min_image(dx: np.ndarray, L: float) -> np.ndarray:
    return dx - L * np.round(dx / L)


def gaussian_field(dims: Sequence[int], G: int, rng: np.random.Generator,
                   amp=(-0.5, 0.5), sigma: Optional[Tuple[float, float]] = None
                   ) -> np.ndarray:
    """Sum of G periodic Gaussians (centres, then widths, then amplitudes)."""
    d = len(dims)
    if sigma is None:
        sigma = (1.5, 4.0) if d == 2 else (2.0, 6.0)
    centres = rng.uniform(0.0, 1.0, size=(G, d)) * np.asarray(dims, dtype=np.float64)
    widths = rng.uniform(sigma[0], sigma[1], size=G)
    amps = rng.uniform(amp[0], amp[1], size=G)
    xs = coords(dims)
    U = np.zeros(int(np.prod(dims)), dtype=np.float64)
    for g in range(G):
        r2 = np.zeros_like(U)
        for a in range(d):
            dx = _min_image(xs[a] - centres[g, a], float(dims[a]))
            r2 += dx * dx
        U += amps[g] * np.exp(-r2 / (2.0 * widths[g] ** 2))
    return U


def pairing_noise(nsites: int, rng: np.random.Generator, scale: float = 1e-3) -> np.ndarray:
    re = rng.standard_normal(nsites)
    im = rng.standard_normal(nsites)
    return scale * (re + 1j * im)


def vortex_2d(dims, delta0: float, heal: float, centre=None, charge: int = 1) -> np.ndarray:
    x, y = coords(dims)[:2]
    cx, cy = centre if centre is not None else (dims[0] // 2, dims[1] // 2)
    dx, dy = x - cx, y - cy
    r = np.hypot(dx, dy)
    theta = charge * np.arctan2(dy, dx)
    return delta0 * np.tanh(r / heal) * np.exp(1j * theta)


def vortex_line_z(dims, delta0: float, heal: float) -> np.ndarray:
    x, y, _ = coords(dims)
    dx, dy = x - dims[0] // 2, y - dims[1] // 2
    rho = np.hypot(dx, dy)
    return delta0 * np.tanh(rho / heal) * np.exp(1j * np.arctan2(dy, dx))


def vortex_ring(dims, delta0: float, radius: float, heal: float = 3.0) -> np.ndarray:
    x, y, z = coords(dims)
    dx, dy, dz = x - dims[0] // 2, y - dims[1] // 2, z - dims[2] // 2
    rho = np.hypot(dx, dy)
    dist = np.hypot(rho - radius, dz)
    phi = np.arctan2(dz, rho - radius)
    return delta0 * np.tanh(dist / heal) * np.exp(1j * phi)


def uniform(dims, U0: float, delta0: complex, mu: float, name="uniform") -> Workload:
    ns = int(np.prod(dims))
    return Workload(name, tuple(int(v) for v in dims),
                    np.full(ns, float(U0)), np.full(ns, complex(delta0)), float(mu))


def random_field(dims, G: int, mu: float, delta_fn, seed: int, name: str) -> Workload:
    rng = _rng(seed)
    dims = tuple(int(v) for v in dims)
    U = gaussian_field(dims, G, rng)
    D = delta_fn(dims) + pairing_noise(int(np.prod(dims)), rng)
    return Workload(name, dims, U, D.astype(np.complex128), float(mu))


# The five workload families of the benchmark, seed = 1000*config + instance.

def tiny_2d(instance: int = 0) -> Workload:
    """2D 16x16, 8 Gaussians, mu=1, single vortex Delta=0.3 tanh(r/2); n=512."""
    return random_field((16, 16), 8, 1.0,
                        lambda d: vortex_2d(d, 0.3, 2.0), 1000 * 1 + instance, "tiny_2d_16x16")


def line_3d(dims=(24, 24, 24), instance: int = 0, config: int = 2) -> Workload:
    """3D vortex line along z, 32 Gaussians, mu=0.8, Delta=0.25 tanh(rho/3)."""
    name = "line_3d_" + "x".join(str(v) for v in dims)
    return random_field(dims, 32, 0.8, lambda d: vortex_line_z(d, 0.25, 3.0),
                        1000 * config + instance, name)


def metric_3d(instance: int = 0) -> Workload:
    """24^3 lattice, n = 27648: the timed configuration."""
    return line_3d((24, 24, 24), instance, config=2)


def precision_3d(instance: int = 0) -> Workload:
    """32x32x24 lattice, n = 49152."""
    return line_3d((32, 32, 24), instance, config=3)


def ring_3d(dims=(32, 32, 32), instance: int = 0) -> Workload:
    """32^3 lattice with a vortex ring of radius 8, n = 65536."""
    name = "ring_3d_" + "x".join(str(v) for v in dims)
    return random_field(dims, 32, 0.8, lambda d: vortex_ring(d, 0.25, 8.0 * dims[0] / 32.0),
                        1000 * 5 + instance, name)


def line_3d_small(dims=(6, 6, 4), instance: int = 0) -> Workload:
    """Same generator as the 3D workloads at a size the oracle solves quickly."""
    return line_3d(dims, instance, config=2)


# ---- SCF instances: harmonic + Gaussian trap and 0-4 vortices (64x64) -------------

@dataclasses.dataclass(frozen=True)
class ScfInstance:
    dims: Tuple[int, ...]
    Vext: np.ndarray      # float64
    theta: np.ndarray     # float64, fixed pairing phase
    mu: float
    seed: int


def scf_instance(instance: int, dims=(64, 64), mu: float = 1.0) -> ScfInstance:
    """Trap V = 0.5 w^2 |r-c|^2 + 1..3 Gaussians, 0..4 vortices of random sign."""
    seed = 1000 * 4 + instance
    rng = _rng(seed)
    Nx, Ny = dims
    scale = Nx / 64.0
    omega = rng.uniform(0.05, 0.15) / scale
    ng = int(rng.integers(1, 4))
    centres = rng.uniform(0.0, 1.0, size=(ng, 2)) * np.array([Nx, Ny], dtype=np.float64)
    widths = rng.uniform(2.0, 6.0, size=ng) * scale
    amps = rng.uniform(-0.5, 0.5, size=ng)
    nv = int(rng.integers(0, 5))
    # vortex cores inside the cloud: within a quarter box of the centre
    vpos = (0.5 + rng.uniform(-0.25, 0.25, size=(nv, 2))) * np.array([Nx, Ny], dtype=np.float64)
    vsign = rng.choice([-1, 1], size=nv)
    x, y = coords(dims)
    cx, cy = Nx / 2.0, Ny / 2.0
    V = 0.5 * omega ** 2 * ((x - cx) ** 2 + (y - cy) ** 2)
    for g in range(ng):
        dx = _min_image(x - centres[g, 0], float(Nx))
        dy = _min_image(y - centres[g, 1], float(Ny))
        V += amps[g] * np.exp(-(dx * dx + dy * dy) / (2.0 * widths[g] ** 2))
    theta = np.zeros_like(x)
    for v in range(nv):
        theta += vsign[v] * np.arctan2(y - vpos[v, 1], x - vpos[v, 0])
    return ScfInstance((Nx, Ny), V, theta, mu, seed)


def scf_instance_3d(instance: int, dims=(16, 16, 8), mu: float = 1.0) -> ScfInstance:
    """3-D trap for the regularised / finite-temperature / multigrid SCF: V =
    0.5 w^2 |r - c|^2 (w ~ U(0.08, 0.16) scaled to a 16-site box) + one
    Gaussian, and a straight vortex line along z through the centre with
    random sign (or none)."""
    seed = 1000 * 6 + instance
    rng = _rng(seed)
    Nx, Ny, Nz = dims
    scale = Nx / 16.0
    omega = rng.uniform(0.08, 0.16) / scale
    centre = rng.uniform(0.0, 1.0, size=3) * np.array([Nx, Ny, Nz], dtype=np.float64)
    width = rng.uniform(1.5, 3.0) * scale
    amp = rng.uniform(-0.5, 0.5)
    sign = int(rng.integers(-1, 2))
    x, y, z = coords(dims)
    cx, cy, cz = Nx / 2.0, Ny / 2.0, Nz / 2.0
    V = 0.5 * omega ** 2 * ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
    dx = _min_image(x - centre[0], float(Nx))
    dy = _min_image(y - centre[1], float(Ny))
    dz = _min_image(z - centre[2], float(Nz))
    V += amp * np.exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * width ** 2))
    theta = sign * np.arctan2(y - cy, x - cx)
    return ScfInstance((Nx, Ny, Nz), V, theta, mu, seed)


def random_hermitian(n: int, seed: int) -> np.ndarray:
    """Dense complex Hermitian test matrix (column-major use is the caller's)."""
    rng = _rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return (A + A.conj().T) / 2.0


def clustered_hermitian(n: int, seed: int):
    """Hermitian Q diag(w) Q^H with a known spectrum holding tight groups:
    pairs 1e-6 and 1e-9 apart and an exactly degenerate triple among uniform
    values in [-5, 5].  Returns (H, w ascending)."""
    rng = _rng(seed)
    w = np.sort(rng.uniform(-5.0, 5.0, n))
    k = n // 5
    w[k], w[k + 1] = 1.0, 1.0 + 1e-6
    w[2 * k], w[2 * k + 1] = -2.0, -2.0 + 1e-9
    w[3 * k] = w[3 * k + 1] = w[3 * k + 2] = 2.5
    w = np.sort(w)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    H = (Q * w) @ Q.conj().T
    return 0.5 * (H + H.conj().T), w


def random_tridiagonal(n: int, seed: int):
    rng = _rng(seed)
    return rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))


# ---- SCF functional constants (a synthetic SLDA-like functional) -----------------
@dataclasses.dataclass(frozen=True)
class ScfParams:
    """Constants of the self-consistency update (plain numbers, no arithmetic).

    U = Vext + B * eps_F(n) (eps_F = pi n in 2D, (3 pi^2 n)^(2/3) / 2 in 3D),
    |Delta| = g |nu| with the phase held fixed, linear mixing alpha, window
    0 < E < Ec, convergence when max|dU|, max|d|Delta|| <= tol.  B and g are
    test constants, not the paper's (its A, B, C are not printed); g makes the
    uniform 2D gas at mu = 1, U = 0 carry Delta = 0.3 on a 64x64 lattice
    (value written by tests/golden/make_scf_constant.py from the oracle).
    T is the temperature of the Fermi function in the densities (0 = ground
    state); regularize = 1 switches on the cut-off regularisation of g (3-D).
    """
    B: float = -0.3
    g: float = 2.356643412040275
    alpha: float = 0.3
    Ec: float = 4.934802200544679   # pi^2 / 2
    tol: float = 1e-6
    max_iter: int = 200
    T: float = 0.0
    regularize: int = 0
