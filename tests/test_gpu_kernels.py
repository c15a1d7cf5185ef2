"""GPU parity of the building-block kernels: assembly and the MFMA GEMM tiles."""
import numpy as np
import pytest

import oracle
from paper_2310_03341_amd import inputs
from tests.gpu_util import need_gpu, to_dev_colmajor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


@pytest.mark.parametrize("w", [inputs.tiny_2d(), inputs.line_3d_small((4, 4, 4)),
                               inputs.line_3d_small((6, 4, 2)),
                               inputs.uniform((8, 8), 0.1, 0.3 + 0.2j, 1.0)],
                         ids=lambda w: w.name)
def test_assemble_matches_oracle(dev, w):
    import torch
    from paper_2310_03341_amd import api
    H = api.assemble(w.dims, torch.from_numpy(w.U).to(dev), torch.from_numpy(w.Delta).to(dev), w.mu)
    torch.cuda.synchronize()
    ref = oracle.assemble_workload(w)
    assert np.abs(H.cpu().numpy() - ref).max() < 1e-13


def test_assemble_metric_size_sampled(dev):
    """24^3 lattice (n = 27648): sampled entries vs the oracle's definition."""
    import torch
    from paper_2310_03341_amd import api
    w = inputs.metric_3d()
    n = w.n
    H = api.assemble(w.dims, torch.from_numpy(w.U).to(dev), torch.from_numpy(w.Delta).to(dev), w.mu)
    rng = np.random.default_rng(0)
    ns = w.nsites
    rows = list(rng.integers(0, n, 600))
    cols = list(rng.integers(0, n, 600))
    # structured nonzeros: diagonal, pairing diagonal, axis neighbours
    for r in rng.integers(0, ns, 100):
        r = int(r)
        rows += [r, r + ns, r, r + ns, r, r]
        cols += [r, r + ns, r + ns, r, (r + 1) % ns, (r + 24 * 24 * 5) % ns]
    ri = torch.tensor(rows, device=dev)
    ci = torch.tensor(cols, device=dev)
    got = H[ri, ci].cpu().numpy()
    ref = oracle.assemble_entries(w.dims, w.U, w.Delta, w.mu, rows, cols)
    assert np.abs(got - ref).max() < 1e-13
    # Hermitian on the samples
    assert np.abs(H[ci, ri].cpu().numpy() - np.conj(got)).max() == 0.0
    del H
    torch.cuda.empty_cache()


SHAPES = [(1, 1, 1), (37, 65, 19), (130, 70, 257), (64, 64, 64), (200, 17, 100),
          (300, 290, 70), (513, 256, 33)]  # the last two take the 128 x 128 tiles (real)


def _op(M, op):
    return M if op == "N" else M.conj().T


@pytest.mark.parametrize("kind", ["z", "c", "d"])
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("N", "C"), ("C", "N"), ("C", "C")])
@pytest.mark.parametrize("shape", SHAPES)
def test_gemm_matches_reference(dev, kind, opA, opB, shape):
    import torch
    from paper_2310_03341_amd import api
    M, N, K = shape
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    real = kind == "d"
    dt = {"z": np.complex128, "c": np.complex64, "d": np.float64}[kind]

    def rnd(r, c):
        X = rng.standard_normal((r, c))
        if not real:
            X = X + 1j * rng.standard_normal((r, c))
        return X.astype(dt)

    A = rnd(M, K) if opA == "N" else rnd(K, M)
    B = rnd(K, N) if opB == "N" else rnd(N, K)
    C = rnd(M, N)
    alpha = 0.75 if real else 0.75 - 0.5j
    beta = -1.25 if real else 0.3 + 1.1j
    ref = alpha * (_op(A.astype(np.complex128), opA) @ _op(B.astype(np.complex128), opB)) \
        + beta * C.astype(np.complex128)
    dA = to_dev_colmajor(A, dev, ld=A.shape[0] + 3)
    dB = to_dev_colmajor(B, dev)
    dC = to_dev_colmajor(C, dev, ld=M + 1)
    fn = {"z": api.zgemm, "c": api.cgemm, "d": api.dgemm}[kind]
    fn(opA, opB, dA, dB, dC, alpha, beta)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    scale = np.sqrt(K) * 4.0
    tol = (2e-15 if kind != "c" else 2e-6) * scale * 4
    assert np.abs(got - ref).max() < tol * max(1.0, np.abs(ref).max() / np.sqrt(K))


def _crand(rng, r, c):
    return rng.standard_normal((r, c)) + 1j * rng.standard_normal((r, c))


@pytest.mark.parametrize("splitk", [1, 2, 3, 7, 64])
@pytest.mark.parametrize("opA,opB,M,N,K", [("N", "N", 130, 64, 1500), ("C", "N", 64, 64, 2500),
                                           ("N", "C", 200, 70, 1039)])
def test_gemm_splitk_full(dev, splitk, opA, opB, M, N, K):
    """The split-K path of the tile GEMM (partial products per K chunk, then
    the reduction kernel) that the stage-1 products use at large n."""
    import torch
    from paper_2310_03341_amd import api
    rng = np.random.default_rng(splitk * 7 + M)
    A = _crand(rng, M, K) if opA == "N" else _crand(rng, K, M)
    B = _crand(rng, K, N) if opB == "N" else _crand(rng, N, K)
    C = _crand(rng, M, N)
    alpha, beta = 0.5 + 0.25j, -0.75 + 0.1j
    ref = alpha * (_op(A, opA) @ _op(B, opB)) + beta * C
    dC = to_dev_colmajor(C, dev, ld=M + 5)
    api.stage_zgemm(0, splitk, opA, opB, to_dev_colmajor(A, dev), to_dev_colmajor(B, dev), dC, alpha, beta)
    torch.cuda.synchronize()
    assert np.abs(dC.cpu().numpy() - ref).max() < 1e-13 * np.sqrt(K) * 4


@pytest.mark.parametrize("splitk", [1, 4, 13])
@pytest.mark.parametrize("M,N", [(700, 64), (1100, 130)])
def test_gemm_splitk_hemm_lower(dev, splitk, M, N):
    """HEMM from the lower triangle (stage 1's A22 V): the strict upper triangle
    of A holds 1e30 garbage, which must not enter the product."""
    import torch
    from paper_2310_03341_amd import api
    rng = np.random.default_rng(M + splitk)
    Hf = _crand(rng, M, M)
    Hf = Hf + Hf.conj().T
    A = np.tril(Hf) + np.triu(np.full((M, M), 1e30 - 1e30j), 1)
    B = _crand(rng, M, N)
    ref = Hf @ B
    dC = to_dev_colmajor(np.zeros((M, N), dtype=np.complex128), dev)
    api.stage_zgemm(2, splitk, "N", "N", to_dev_colmajor(A, dev), to_dev_colmajor(B, dev), dC, 1.0, 0.0)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    assert np.abs(got - ref).max() < 1e-13 * np.sqrt(M) * 8


def test_gemm_lower_tiles(dev):
    """Lower-tile mode writes the 64 x 64 tiles on and below the diagonal only;
    it refuses a split of K."""
    import torch
    from paper_2310_03341_amd import api
    rng = np.random.default_rng(5)
    M, K = 200, 90
    A, B = _crand(rng, M, K), _crand(rng, M, K)
    C = _crand(rng, M, M)
    ref = -1.0 * (A @ B.conj().T) + C
    dC = to_dev_colmajor(C, dev)
    api.stage_zgemm(1, 1, "N", "C", to_dev_colmajor(A, dev), to_dev_colmajor(B, dev), dC, -1.0, 1.0)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    I, J = np.meshgrid(np.arange(M) // 64, np.arange(M) // 64, indexing="ij")
    low = I >= J
    assert np.abs(got[low] - ref[low]).max() < 1e-13 * 40
    assert np.abs(got[~low] - C[~low]).max() == 0.0
    with pytest.raises(api.BdgError):
        api.stage_zgemm(1, 2, "N", "C", to_dev_colmajor(A, dev), to_dev_colmajor(B, dev), dC, -1.0, 1.0)


def test_complex_gemm_refuses_plain_transpose(dev):
    from paper_2310_03341_amd import api
    A = to_dev_colmajor(np.eye(4, dtype=np.complex128), dev)
    with pytest.raises(api.BdgError):
        api.zgemm("T", "N", A, A, A)
