"""bdg_eigh1 (one-stage FP64 solver, real symmetric and complex Hermitian)
against the oracle: eigenvalues within 1e-10 of the spectral width, residual
and Gram defect of every pair on the host in FP64 within 1e-12."""
import numpy as np
import pytest

import oracle
from paper_2310_03341_amd import inputs
from tests.gpu_util import need_gpu, to_dev_colmajor

pytestmark = pytest.mark.gpu

EIG_TOL = 1e-10
VEC_TOL = 1e-12


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _check(H, W, Z, ref, idx=None):
    width = ref[-1] - ref[0] if ref.size > 1 else max(1.0, abs(ref[0]))
    want = ref if idx is None else ref[idx]
    assert W.size == want.size
    assert np.abs(W - want).max() <= EIG_TOL * width
    normH = max(np.abs(ref).max(), 1e-300)
    res = np.linalg.norm(H @ Z - Z * W, axis=0).max() / normH
    gram = np.abs(Z.conj().T @ Z - np.eye(Z.shape[1])).max()
    assert res <= VEC_TOL and gram <= VEC_TOL, (res, gram)


def _solve(dev, H, lo=-np.inf, hi=np.inf, ld=None):
    import torch
    from paper_2310_03341_amd import api
    A = to_dev_colmajor(H, dev, ld=ld)
    W, Z, rep = api.eigh1(A, lo, hi)
    torch.cuda.synchronize()
    return W.cpu().numpy(), Z.cpu().numpy(), rep


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 65, 130, 300, 517])
@pytest.mark.parametrize("real", [True, False])
def test_eigh1_random_matches_oracle(dev, n, real):
    H = inputs.random_hermitian(n, 40 + n)
    if real:
        H = np.ascontiguousarray(H.real)
    print("eigh1 n=%d real=%s" % (n, real), flush=True)
    ref = oracle.eigh_hqr(H.astype(np.complex128), vectors=False)[0]
    W, Z, _ = _solve(dev, H)
    _check(H, W, Z, ref)


@pytest.mark.parametrize("real", [True, False])
def test_eigh1_bdg_matrix_window_and_ld(dev, real):
    """The 16x16 vortex BdG matrix (complex), or the same fields with a real
    gap (real symmetric), a window inside the spectrum, lda > n."""
    w = inputs.tiny_2d()
    if real:
        w = inputs.Workload(w.name, w.dims, w.U, np.abs(w.Delta).astype(np.complex128), w.mu)
    H = oracle.assemble_workload(w)
    if real:
        assert np.abs(H.imag).max() == 0.0
        H = np.ascontiguousarray(H.real)
    ref = oracle.eigh_hqr(H.astype(np.complex128), vectors=False)[0]
    lo, hi = 0.05, 2.0
    idx = np.flatnonzero((ref >= lo) & (ref <= hi))
    W, Z, _ = _solve(dev, H, lo, hi, ld=H.shape[0] + 7)
    _check(H, W, Z, ref, idx)


def test_eigh1_clustered_and_degenerate(dev):
    """Exact degeneracies and pairs 1e-6 / 1e-9 apart (complex)."""
    H, wtrue = inputs.clustered_hermitian(400, 5)
    W, Z, _ = _solve(dev, H)
    _check(H, W, Z, wtrue)


def test_eigh1_n2048_both_types(dev):
    """n = 2048 (2-D 32x32 vortex lattice): many panels, long hemv tile columns."""
    w = inputs.random_field((32, 32), 8, 1.0, lambda d: inputs.vortex_2d(d, 0.3, 2.0), 1007, "mid_2d")
    H = oracle.assemble_workload(w)
    ref = oracle.eigh_hqr(H, vectors=False)[0]
    W, Z, rep = _solve(dev, H)
    print("complex n=2048: %.1f ms (trd %.1f, D&C %.1f, back %.1f)" % (
        rep.stage_ms[7], rep.stage_ms[0], rep.stage_ms[2], rep.stage_ms[4]))
    _check(H, W, Z, ref)
    wr = inputs.Workload(w.name, w.dims, w.U, np.abs(w.Delta).astype(np.complex128), w.mu)
    Hr = np.ascontiguousarray(oracle.assemble_workload(wr).real)
    refr = oracle.eigh_hqr(Hr.astype(np.complex128), vectors=False)[0]
    W, Z, rep = _solve(dev, Hr)
    print("real n=2048: %.1f ms" % rep.stage_ms[7])
    _check(Hr, W, Z, refr)
