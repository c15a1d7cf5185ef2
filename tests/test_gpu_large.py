"""Parity of bdg_eigh at the sizes its kernels run at.

* n = 2048 (2D 32x32 vortex lattice): every stage takes its large-size path
  (stage-1 products split K over several workgroups and reduce the partial
  sums); eigenvalues against the oracle's Householder + QL within 1e-10 of the
  width, residual and Gram defect of every pair computed on the host in FP64.
* The timed workload, n = 27648 (24^3 vortex line), full spectrum in FP64
  with the particle-hole mirror as the benchmark runs it: the oracle cannot
  diagonalise it on the CPU, so the checks are what holds at any size --
  residuals ||H z - w z|| / ||H||_2 of 256 sampled eigenvectors from the
  oracle's matrix-free H (FP64, host), their Gram matrix, the particle-hole
  symmetry of the spectrum, tr H = sum w = 0 and ||H||_F^2 = sum w^2 with
  ||H||_F^2 from its definition.
* Uniform fields at n = 27648 and n = 49152 (32x32x24, where n^2 exceeds 2^31
  and every index runs in 64 bits): all eigenvalues against the closed form
  +-sqrt((eps_k + U0 - mu)^2 + |Delta0|^2), sampled residuals and Gram.
* Leading dimensions larger than n.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2310_03341_amd import inputs
from tests.gpu_util import need_gpu, to_dev_colmajor
from tests.test_oracle import uniform_spectrum

pytestmark = pytest.mark.gpu

EIG_TOL = 1e-10
VEC_TOL = 1e-12


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _host_check(H, W, Z):
    normH = np.abs(W).max()
    res = np.linalg.norm(H @ Z - Z * W, axis=0).max() / normH
    gram = np.abs(Z.conj().T @ Z - np.eye(Z.shape[1])).max()
    return res, gram


def mid_2d():
    return inputs.random_field((32, 32), 8, 1.0, lambda d: inputs.vortex_2d(d, 0.3, 2.0), 1000 * 1 + 7,
                               "mid_2d_32x32")


@pytest.mark.parametrize("precision,ph", [(0, 0), (0, 1), (1, 1)])
def test_eigh_n2048_matches_oracle(dev, precision, ph):
    import torch
    from paper_2310_03341_amd import api
    w = mid_2d()
    H = oracle.assemble_workload(w)
    ref = oracle.eigh_hqr(H, vectors=False)[0]
    A = to_dev_colmajor(H, dev)
    W, Z = api.eigh(A, opts=api.make_opts(precision=precision, ph_mirror=ph))
    torch.cuda.synchronize()
    W, Z = W.cpu().numpy(), Z.cpu().numpy()
    assert np.abs(W - ref).max() <= EIG_TOL * (ref[-1] - ref[0])
    res, gram = _host_check(H, W, Z)
    assert res <= VEC_TOL and gram <= VEC_TOL, (res, gram)


def test_eigh_leading_dimensions(dev):
    """lda = n + 20 and ldz = n + 10 (column-major views into wider buffers)."""
    import torch
    from paper_2310_03341_amd import api
    n = 300
    H = inputs.random_hermitian(n, 31)
    ref = oracle.eigh_hqr(H, vectors=False)[0]
    for precision in (0, 1):
        A = to_dev_colmajor(H, dev, ld=n + 20)
        Z = api.colmajor(n, n, torch.complex128, dev, ld=n + 10)
        Z.fill_(7.0)
        W, Zv = api.Solver(n, api.make_opts(precision=precision), dev)(A, Z=Z)
        torch.cuda.synchronize()
        assert A.stride(1) == n + 20 and Zv.stride(1) == n + 10
        W, Zh = W.cpu().numpy(), Zv.cpu().numpy()
        assert np.abs(W - ref).max() <= EIG_TOL * (ref[-1] - ref[0])
        res, gram = _host_check(H, W, Zh)
        assert res <= VEC_TOL and gram <= VEC_TOL, (precision, res, gram)


def _frobenius2(w):
    """||H||_F^2 of eq. (stHpsi) from its definition: 2 ||h||_F^2 + 2 sum |Delta|^2,
    h = sum_d T_d (along axis d) + diag(U - mu); every site has N_d - 1
    neighbours along axis d, each coupled by an off-diagonal entry of T_d."""
    T = [oracle.kinetic_1d(N) for N in w.dims]
    diag = sum(t[0, 0] for t in T) + w.U - w.mu
    off = sum(float(np.sum(t ** 2) - N * t[0, 0] ** 2) / N for t, N in zip(T, w.dims))
    h2 = float(np.sum(diag ** 2)) + w.nsites * off
    return 2.0 * h2 + 2.0 * float(np.sum(np.abs(w.Delta) ** 2))


def _solve_sampled(dev, w, nsample=256, seed=0):
    """FP64 solve of the full spectrum (particle-hole mirror on); returns all
    eigenvalues and nsample eigenvectors (host), chosen at the spectrum's ends,
    around E = 0 and at random."""
    import torch
    from paper_2310_03341_amd import api
    n = w.n
    print("solve n=%d (%s)" % (n, w.name), flush=True)
    H = api.assemble(w.dims, torch.from_numpy(w.U).to(dev), torch.from_numpy(w.Delta).to(dev), w.mu)
    solver = api.Solver(n, api.make_opts(ph_mirror=1), dev)
    W, Z = solver(H)
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    h = n // 2
    idx = np.unique(np.r_[0, 1, 2, h - 3:h + 3, n - 3:n, rng.choice(n, nsample, replace=False)])[:nsample]
    Zs = Z[:, torch.from_numpy(idx).to(dev)].cpu().numpy()
    Wh = W.cpu().numpy()
    t = solver.report.stage_ms[7] / 1e3
    del solver, H, Z, W
    torch.cuda.empty_cache()
    print("  solved in %.2f s" % t, flush=True)
    return Wh, idx, Zs


def _check_sampled(w, W, idx, Zs):
    normH = np.abs(W).max()
    R = oracle.apply_h(w.dims, w.U, w.Delta, w.mu, Zs) - Zs * W[idx]
    res = np.linalg.norm(R, axis=0).max() / normH
    gram = np.abs(Zs.conj().T @ Zs - np.eye(idx.size)).max()
    return res, gram


@pytest.mark.parametrize("which", ["uniform", "metric"])
def test_eigh_metric_size(dev, which):
    if which == "uniform":
        w = inputs.uniform((24, 24, 24), 0.05, 0.25 * np.exp(0.7j), 0.8, "uniform_24x24x24")
    else:
        w = inputs.metric_3d()
    W, idx, Zs = _solve_sampled(dev, w)
    width = W[-1] - W[0]
    assert np.all(np.diff(W) >= 0)
    assert np.abs(W + W[::-1]).max() <= 1e-12 * width
    if which == "uniform":
        ref = uniform_spectrum(w.dims, 0.05, 0.25 * np.exp(0.7j), 0.8)
        assert np.abs(W - ref).max() <= EIG_TOL * width
    # tr H = 0 and sum w^2 = ||H||_F^2
    assert abs(W.sum()) <= 1e-12 * w.n * np.abs(W).max()
    f2 = _frobenius2(w)
    assert abs(np.sum(W ** 2) - f2) <= 1e-12 * f2
    res, gram = _check_sampled(w, W, idx, Zs)
    print("  sampled residual %.2e gram %.2e" % (res, gram))
    assert res <= VEC_TOL and gram <= VEC_TOL, (res, gram)


def test_eigh_64bit_indices_uniform(dev):
    """32x32x24 lattice, n = 49152: n^2 = 2.4e9 > 2^31."""
    w = inputs.uniform((32, 32, 24), -0.1, 0.2 + 0.15j, 0.8, "uniform_32x32x24")
    W, idx, Zs = _solve_sampled(dev, w)
    ref = uniform_spectrum(w.dims, -0.1, 0.2 + 0.15j, 0.8)
    width = ref[-1] - ref[0]
    assert np.abs(W - ref).max() <= EIG_TOL * width
    res, gram = _check_sampled(w, W, idx, Zs)
    print("  sampled residual %.2e gram %.2e" % (res, gram))
    assert res <= VEC_TOL and gram <= VEC_TOL, (res, gram)
