"""Multigrid start of the SLDA self-consistency (all field arithmetic on the GPU).

The paper reaches its largest static states by solving on coarser lattices
first, each solution starting the iteration on the next finer lattice (sec.
"Performance of the Matrix Diagonalization Algorithm": N = 60, 80, 100).  The
library's unit of length is the lattice spacing on every level, so the coarse
level with spacing s fine spacings is the same physical problem in rescaled
units: lengths / s, energies * s^2 (Vext, mu, T, the fields U and |Delta|),
densities * s^d, couplings g * s^(2-d); its cut-off Ec stays pi^2/2 of its own
lattice.  bdg_regrid samples the fine inputs at every s-th site (injection)
and carries the converged coarse fields back by trigonometric interpolation,
with the energy rescaling folded in.  The coarse cut-off is lower than the
fine one (pi^2/2 / s^2 in fine units), so without the cut-off regularisation
(3-D) the coarse gap is the solution of a different problem and only
approximately right.
"""
from __future__ import annotations

import dataclasses

import torch

from . import api, inputs
from .learned_start import UNIFORM_DELTA, run_scf


def coarse_params(p: inputs.ScfParams, s: int, ndim: int) -> inputs.ScfParams:
    """The SCF constants of the level with s times the spacing (rescaled units)."""
    return dataclasses.replace(p, g=p.g * float(s) ** (2 - ndim), T=p.T * s * s)


def multigrid_start(inst: inputs.ScfInstance, p: inputs.ScfParams, dev, s: int = 2, log=None):
    """Solve the instance on the lattice coarser by s (uniform start there) and
    return the fine-lattice start fields (U, |Delta|) and the coarse iteration count."""
    dims = tuple(int(v) for v in inst.dims)
    if any(N % (2 * s) for N in dims):
        raise ValueError("every lattice size must be a multiple of 2 s")
    dc = tuple(N // s for N in dims)
    Vext = torch.from_numpy(inst.Vext).to(dev)
    theta = torch.from_numpy(inst.theta).to(dev)
    Vc = api.regrid(dims, Vext, dc, scale=float(s * s))
    thc = api.regrid(dims, theta, dc, scale=1.0)
    pc = coarse_params(p, s, len(dims))
    st = api.ScfStepper(dc, Vc, thc, inst.mu * s * s, pc)
    Uc = Vc.clone()
    Dc = torch.full_like(Vc, UNIFORM_DELTA * s * s)
    iters, ok, _ = run_scf(st, Uc, Dc, pc)
    if log:
        log("coarse %s: %d iterations (%s)" % ("x".join(map(str, dc)), iters, "ok" if ok else "not converged"))
    U = api.regrid(dc, Uc, dims, scale=1.0 / (s * s))
    D = api.regrid(dc, Dc, dims, scale=1.0 / (s * s))
    return U, D, iters
