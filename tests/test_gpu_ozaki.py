"""bdg_gemm_int8 (FP64 products emulated on the INT8 matrix cores) against the
oracle's slice arithmetic and the exact product's error bound."""
import numpy as np
import pytest

from oracle import ozaki
from tests.gpu_util import need_gpu, to_dev_colmajor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _op(X, op):
    return X if op == "N" else X.conj().T


def _run(dev, opA, opB, A, B, C0, alpha, beta, slices):
    import torch
    from paper_2310_03341_amd import api
    Ad, Bd, Cd = to_dev_colmajor(A, dev), to_dev_colmajor(B, dev), to_dev_colmajor(C0, dev)
    api.gemm_int8(opA, opB, Ad, Bd, Cd, alpha, beta, slices)
    torch.cuda.synchronize()
    return Cd.cpu().numpy()


def _scale_matrix(opA_A, opB_B):
    """2^(e_r + e_c) of the error bound (real and imaginary parts together)."""
    def ex(X, axis):
        m = np.maximum(np.abs(X.real), np.abs(X.imag)).max(axis=axis)
        e = np.zeros(m.shape)
        nz = m > 0
        e[nz] = np.frexp(m[nz])[1] + 1
        return e
    return np.ldexp(1.0, (ex(opA_A, 1)[:, None] + ex(opB_B, 0)[None, :]).astype(int))


@pytest.mark.parametrize("M,N,K", [(64, 64, 64), (1, 1, 1), (70, 33, 129), (200, 150, 300)])
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("C", "N"), ("N", "C"), ("C", "C")])
def test_real_int8_gemm_matches_oracle(dev, M, N, K, opA, opB):
    rng = np.random.default_rng(M + 3 * N + 7 * K)
    A = rng.standard_normal((M, K) if opA == "N" else (K, M)) * 10.0 ** rng.uniform(-4, 4)
    B = rng.standard_normal((K, N) if opB == "N" else (N, K))
    A[0, :] *= 1e-9  # a line with a very different scale
    C0 = rng.standard_normal((M, N))
    print("real int8 gemm %s%s %dx%dx%d" % (opA, opB, M, N, K), flush=True)
    got = _run(dev, opA, opB, A, B, C0, 1.5, -0.5, 8)
    oa, ob = _op(A, opA), _op(B, opB)
    emu = 1.5 * ozaki.gemm_real(oa, ob, 8) - 0.5 * C0
    sc = _scale_matrix(oa, ob)
    # same integers, summed in FP64 in another order
    assert np.all(np.abs(got - emu) <= 1.5 * 4 * K * 2.0 ** -52 * sc * 2.0 ** -7 + 1e-300)
    exact = 1.5 * (oa @ ob) - 0.5 * C0
    assert np.all(np.abs(got - exact) <= 1.5 * ozaki.error_bound(oa, ob, 8) + 8 * K * 2.0 ** -53 * sc + 1e-14 * np.abs(C0))


@pytest.mark.parametrize("opA,opB", [("C", "N"), ("N", "N"), ("N", "C")])
@pytest.mark.parametrize("slices", [4, 8])
def test_complex_int8_gemm(dev, opA, opB, slices):
    rng = np.random.default_rng(slices)
    M, N, K = 96, 80, 200
    A = rng.standard_normal((M, K) if opA == "N" else (K, M)) + 1j * rng.standard_normal((M, K) if opA == "N" else (K, M))
    B = rng.standard_normal((K, N) if opB == "N" else (N, K)) + 1j * rng.standard_normal((K, N) if opB == "N" else (N, K))
    C0 = np.zeros((M, N), dtype=np.complex128)
    got = _run(dev, opA, opB, A, B, C0, 1.0 + 0.5j, 0.0, slices)
    oa, ob = _op(A, opA), _op(B, opB)
    emu = (1.0 + 0.5j) * ozaki.gemm_complex(oa, ob, slices)
    sc = _scale_matrix(oa, ob)
    assert np.all(np.abs(got - emu) <= 8 * 2 * K * 2.0 ** -52 * sc)
    exact = (1.0 + 0.5j) * (oa @ ob)
    err = np.abs(got - exact)
    bound = 1.2 * 2 * (2 * ozaki.error_bound(np.abs(oa), np.abs(ob), slices)) + 16 * K * 2.0 ** -53 * sc
    assert np.all(err <= bound)
    if slices == 8:
        assert err.max() <= 1e-13 * np.abs(exact).max()
    else:
        assert err.max() > 1e-10 * np.abs(exact).max()  # 4 slices: visibly coarser
