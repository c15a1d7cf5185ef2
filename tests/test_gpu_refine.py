"""bdg_refine (Ogita-Aishima FP64 refinement) against the oracle's step.

One GPU step from an FP32-rounded basis is compared with
``oracle.refine.oa_step_window`` (same close-pair rule, same Rayleigh-Ritz
inside clusters) on a spectrum with an exactly degenerate triple and pairs
1e-6 and 1e-9 apart:

* eigenvalues of the step within 1e-13 ||H||_2;
* columns outside the oracle's clusters and outside near-degenerate groups
  element by element within 1e-10.  Two FP64 evaluations of the step that only
  sum in another order differ by up to 2e-12 there, while the step itself
  moves entries by ~1e-7;
* columns inside a cluster, or in a group of step eigenvalues less than
  1e-6 ||H||_2 apart, are unique only as a subspace: an exact triple has no
  preferred basis, and the first-order coefficient of a pair with gap g
  carries a rounding error of about u ||H||_2 / g (7e-8 for the 1e-9 pair,
  which the close-pair rule need not flag: its coefficient is small, just not
  well determined), so their orthogonal projectors are compared instead
  (agreement ~1e-14 between two such evaluations).

Then the full refinement (default step count) from FP32 must reach the FP64
targets, checked on the host in numpy, and the mixed-precision eigensolver
must cut its window on refined eigenvalues.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import refine as oref
from paper_2310_03341_amd import inputs
from tests.gpu_util import need_gpu, to_dev_colmajor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _fp32_basis(H):
    W0, Z0 = np.linalg.eigh(H)
    return W0.astype(np.float32).astype(np.float64), Z0.astype(np.complex64).astype(np.complex128)


def _gpu_refine(dev, H, lam, X, i0, m, steps):
    import torch
    from paper_2310_03341_amd import api
    Hd = to_dev_colmajor(H, dev)
    Xd = to_dev_colmajor(X, dev)
    lamd = torch.from_numpy(lam).to(dev)
    W, rep = api.refine(Hd, lamd, Xd, i0, m, api.make_opts(refine_max_iter=steps))
    torch.cuda.synchronize()
    return W.cpu().numpy(), Xd.cpu().numpy(), rep


@pytest.mark.parametrize("seed,i0,m", [(21, 0, 512), (23, 0, 512), (21, 100, 200), (23, 350, 120)])
def test_refine_step_matches_oracle(dev, seed, i0, m):
    n = 512
    H, wtrue = inputs.clustered_hermitian(n, seed)
    lam, X = _fp32_basis(H)
    normH = np.abs(lam).max()
    cols = np.arange(i0, i0 + m)
    XW_ref, lW_ref, clusters = oref.oa_step_window(H, X, lam, cols, normH, return_clusters=True)
    W, Xg, rep = _gpu_refine(dev, H, lam, X, i0, m, steps=1)
    assert rep.refine_iters == 1
    assert np.abs(W - lW_ref).max() <= 1e-13 * normH
    XW = Xg[:, cols]
    # the columns the step did not touch are unchanged
    rest = np.setdiff1d(np.arange(n), cols)
    if rest.size:
        assert np.abs(Xg[:, rest] - X[:, rest]).max() == 0.0
    in_cluster = np.zeros(m, dtype=bool)
    for J in clusters:
        in_cluster[J] = True
    # the exact triple is a cluster whenever the window holds it
    triple = np.flatnonzero(wtrue == 2.5)
    if np.all((triple >= i0) & (triple < i0 + m)):
        assert in_cluster[triple - i0].all()
    groups = [J for J in clusters]
    order = np.argsort(lW_ref, kind="stable")
    cur = [order[0]]
    for a, b in zip(order[:-1], order[1:]):
        if lW_ref[b] - lW_ref[a] <= 1e-6 * normH:
            cur.append(b)
            continue
        if len(cur) > 1:
            groups.append(np.array(cur))
        cur = [b]
    if len(cur) > 1:
        groups.append(np.array(cur))
    # merge groups that share a column (a cluster inside a near-degenerate run)
    label = np.arange(m)
    for J in groups:
        label[np.isin(label, label[J])] = label[J[0]]
    groups = [np.flatnonzero(label == k) for k in np.unique(label) if np.sum(label == k) > 1]
    grouped = np.zeros(m, dtype=bool)
    for J in groups:
        grouped[J] = True
        P = XW[:, J] @ XW[:, J].conj().T
        Pr = XW_ref[:, J] @ XW_ref[:, J].conj().T
        assert np.abs(P - Pr).max() <= 1e-10, J
    free = ~grouped
    assert np.abs(XW[:, free] - XW_ref[:, free]).max() <= 1e-10
    # the step moved the basis by about the FP32 error
    assert np.abs(XW_ref[:, free] - X[:, cols][:, free]).max() > 1e-9


@pytest.mark.parametrize("window", ["all", "sub"])
def test_refine_reaches_fp64(dev, window):
    """Default steps from an FP32 basis of the 16x16 vortex matrix: eigenvalues
    within 1e-10 of the width of the oracle's, residual and Gram defect of the
    refined columns (host FP64) within 1e-12."""
    H = oracle.assemble_workload(inputs.tiny_2d())
    n = H.shape[0]
    ref = oracle.eigh_hqr(H, vectors=False)[0]
    lam, X = _fp32_basis(H)
    i0, m = (0, n) if window == "all" else (256, 150)
    W, Xg, rep = _gpu_refine(dev, H, lam, X, i0, m, steps=0)
    Z = Xg[:, i0:i0 + m]
    normH = np.abs(ref).max()
    assert np.abs(np.sort(W) - ref[i0:i0 + m]).max() <= 1e-10 * (ref[-1] - ref[0])
    res = np.linalg.norm(H @ Z - Z * W, axis=0).max() / normH
    gram = np.abs(Z.conj().T @ Z - np.eye(m)).max()
    assert res <= 1e-12 and gram <= 1e-12, (res, gram, rep.refine_iters)
    assert 1 <= rep.refine_iters <= 4


def test_refine_empty_window(dev):
    H = inputs.random_hermitian(40, 3)
    lam, X = _fp32_basis(H)
    W, Xg, rep = _gpu_refine(dev, H, lam, X, 10, 0, steps=0)
    assert W.size == 0 and np.abs(Xg - X).max() == 0.0


@pytest.mark.parametrize("seed", [21, 23, 25])
def test_mixed_window_is_cut_on_refined_eigenvalues(dev, seed):
    """Window edges 1e-10 from eigenvalues: far below the FP32 stages' error,
    so only a cut made after refinement returns exactly the eigenvalues inside."""
    from paper_2310_03341_amd import api
    n = 240
    H, w = inputs.clustered_hermitian(n, seed)
    a, b = 37, 181
    emin, emax = w[a] - 1e-10, w[b + 1] - 1e-10
    A = to_dev_colmajor(H, dev)
    solver = api.Solver(n, api.make_opts(precision=api.BDG_FP32_REFINED), dev)
    W, Z = solver(A, emin, emax)
    W = W.cpu().numpy()
    Z = Z.cpu().numpy()
    assert W.size == b + 1 - a
    assert np.abs(W - w[a:b + 1]).max() <= 1e-12 * (w[-1] - w[0])
    res = np.linalg.norm(H @ Z - Z * W, axis=0).max() / np.abs(w).max()
    assert res <= 1e-12


def test_mixed_window_max_pairs(dev):
    """A window smaller than max_pairs runs in the reduced workspace; one that
    needs more columns than max_pairs allows is refused with the count."""
    from paper_2310_03341_amd import api
    H = oracle.assemble_workload(inputs.tiny_2d())
    n = H.shape[0]
    Ec = math.pi ** 2 / 2
    Wr, _ = oracle.eigh(H, 0.0, Ec)
    opts = api.make_opts(precision=api.BDG_FP32_REFINED, max_pairs=Wr.size)
    assert api.eigh_workspace(n, opts) < api.eigh_workspace(n, api.make_opts(precision=1))
    W, Z = api.Solver(n, opts, dev)(to_dev_colmajor(H, dev), 0.0, Ec)
    assert W.numel() == Wr.size
    assert np.abs(W.cpu().numpy() - Wr).max() <= 1e-10 * Ec
    small = api.make_opts(precision=api.BDG_FP32_REFINED, max_pairs=10)
    with pytest.raises(api.BdgError) as ei:
        api.Solver(n, small, dev)(to_dev_colmajor(H, dev), 0.0, Ec)
    assert ei.value.code == 4
