"""GPU parity of each stage of the two-stage solver against the CPU oracle.

Stage outputs are compared through what the method must preserve: the
spectrum (oracle eigensolvers on the band / tridiagonal / dense matrix),
orthonormality of the accumulated transformations and residuals.
"""
import numpy as np
import pytest

import oracle
from paper_2310_03341_amd import inputs
from tests.gpu_util import need_gpu, to_dev_colmajor

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def band_to_dense(AB: np.ndarray, band: int) -> np.ndarray:
    """AB[j, d] = B(j + d, j) for d <= band -> dense Hermitian B."""
    n = AB.shape[0]
    B = np.zeros((n, n), dtype=np.complex128)
    for dd in range(band + 1):
        idx = np.arange(n - dd)
        B[idx + dd, idx] = AB[idx, dd]
    B = B + np.tril(B, -1).conj().T
    return B


def tridiag(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


# ---------------------------------------------------------------- D&C
def _tridiag_cases():
    rng = np.random.default_rng(5)
    cases = []
    for n in (1, 2, 3, 7, 32, 33, 64, 100, 257, 1000):
        cases.append(("rand%d" % n, rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))))
    n = 300
    cases.append(("toeplitz", np.full(n, 2.0), np.ones(n - 1)))
    m = 21
    w = np.abs(np.arange(m) - m // 2).astype(float)
    e = np.ones(8 * m - 1)
    e[m - 1::m] = 1e-9
    cases.append(("glued_wilkinson", np.concatenate([w] * 8), e))
    d = np.repeat([1.0, 2.0, 3.0], 50)
    e = np.zeros(149)
    cases.append(("decoupled_degenerate", d, e))
    e = np.full(199, 1e-12)
    cases.append(("tiny_coupling", rng.standard_normal(200), e))
    # merges wider than one staged chunk of the deflation scan, and more
    # deflated columns than its LDS window (many repeated diagonal values)
    n = 4500
    cases.append(("rand4500", rng.standard_normal(n), rng.standard_normal(n - 1)))
    cases.append(("repeated4500", np.round(rng.uniform(0.0, 4.0, n), 1), 1e-3 * rng.standard_normal(n - 1)))
    return cases


@pytest.mark.parametrize("name,d,e", _tridiag_cases(), ids=lambda c: c if isinstance(c, str) else "")
def test_stedc_matches_oracle(dev, name, d, e):
    import torch
    from paper_2310_03341_amd import api
    n = d.size
    W, Q = api.stage_stedc(torch.from_numpy(d).to(dev), torch.from_numpy(e).to(dev))
    torch.cuda.synchronize()
    W = W.cpu().numpy()
    Q = Q.cpu().numpy()
    ref = oracle.tridiag_eigh(d, e, vectors=False)
    width = max(ref[-1] - ref[0], 1.0)
    assert np.all(np.diff(W) >= 0)
    assert np.abs(W - ref).max() <= 1e-13 * width * max(1, np.sqrt(n) / 4)
    T = tridiag(d, e)
    normT = max(np.abs(ref).max(), 1e-300)
    assert np.abs(T @ Q - Q * W).max() / normT < 1e-13
    assert np.abs(Q.T @ Q - np.eye(n)).max() < 1e-13


# ---------------------------------------------------------------- stage 1
# n = 1200 and 2048: the panels' products split K over several workgroups
# (K chunks of >= 512) and sum the partial products in a second kernel
@pytest.mark.parametrize("kind,n,band", [("rand", 130, 64), ("rand", 300, 32), ("tiny2d", 512, 64),
                                         ("rand", 97, 16), ("uniform", 128, 64), ("rand", 1200, 64),
                                         ("mid2d", 2048, 64)])
def test_he2hb_preserves_spectrum(dev, kind, n, band):
    import torch
    from paper_2310_03341_amd import api
    if kind == "rand":
        H = inputs.random_hermitian(n, seed=n)
    elif kind == "tiny2d":
        H = oracle.assemble_workload(inputs.tiny_2d())
    elif kind == "mid2d":
        from tests.test_gpu_large import mid_2d
        H = oracle.assemble_workload(mid_2d())
    else:
        H = oracle.assemble_workload(inputs.uniform((8, 8), 0.1, 0.3, 1.0))
    A = to_dev_colmajor(H, dev)
    AB, T1 = api.stage_he2hb(A, band)
    torch.cuda.synchronize()
    B = band_to_dense(AB.cpu().numpy(), band)
    ref = oracle.eigh_hqr(H, vectors=False)[0]
    got = oracle.eigh_hqr(B, vectors=False)[0]
    width = ref[-1] - ref[0]
    assert np.abs(got - ref).max() < 1e-12 * width
    # Q1 from the reflectors: Q1 = bt1(I); Q1 unitary and Q1 B Q1^H = H
    I = to_dev_colmajor(np.eye(n, dtype=np.complex128), dev)
    Q1 = api.stage_bt1(A, T1, I, band)
    torch.cuda.synchronize()
    Q1 = Q1.cpu().numpy()
    assert np.abs(Q1.conj().T @ Q1 - np.eye(n)).max() < 1e-13
    assert np.abs(Q1 @ B @ Q1.conj().T - H).max() < 1e-12 * np.abs(H).max() * np.sqrt(n)


# ---------------------------------------------------------------- stage 2 + BT2
def random_band(n, band, seed):
    rng = np.random.default_rng(seed)
    AB = np.zeros((n, 2 * band + 2), dtype=np.complex128)
    for dd in range(band + 1):
        v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        if dd == 0:
            v = v.real.astype(np.complex128)
        v[n - dd:] = 0
        AB[:, dd] = v
    return AB


@pytest.mark.parametrize("n,band", [(5, 4), (64, 8), (200, 16), (301, 64), (130, 64), (513, 32), (250, 48),
                                    (2000, 64)])
def test_hb2st_and_bt2(dev, n, band):
    import torch
    from paper_2310_03341_amd import api
    ABh = random_band(n, band, seed=n + band)
    B = band_to_dense(ABh, band)
    AB = torch.from_numpy(ABh).to(dev)
    d, e, V2, tau2, voff = api.stage_hb2st(AB, band)
    torch.cuda.synchronize()
    dh, eh = d.cpu().numpy(), e.cpu().numpy()[: n - 1]
    ref = oracle.eigh_hqr(B, vectors=False)[0]
    got = oracle.tridiag_eigh(dh, np.abs(eh), vectors=False)
    width = ref[-1] - ref[0]
    assert np.abs(got - ref).max() < 1e-12 * width
    # eigenvectors of B via GPU D&C + BT2
    ea = torch.from_numpy(np.abs(eh).copy()).to(dev)
    W, Y = api.stage_stedc(d, ea)
    Wh = W.cpu().numpy()
    assert np.abs(Wh - ref).max() < 1e-12 * width
    # both routes of the back-transformation 2 (row-major copy of Z, and in
    # place on the column-major Z when the workspace has no room for the copy)
    Zs = []
    for rowmajor in (True, False):
        Z = api.stage_bt2(e, Y, 0, n, V2, tau2, voff, band, rowmajor=rowmajor)
        torch.cuda.synchronize()
        Zh = Z.cpu().numpy()
        assert np.abs(B @ Zh - Zh * Wh).max() < 1e-12 * np.abs(ref).max(), rowmajor
        assert np.abs(Zh.conj().T @ Zh - np.eye(n)).max() < 1e-12, rowmajor
        Zs.append(Zh)
    assert np.abs(Zs[0] - Zs[1]).max() < 1e-12


_CHILD_BT2 = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[2])
from paper_2310_03341_amd import api
d = sys.argv[1]
dev = torch.device("cuda:0")
ld = lambda k: torch.from_numpy(np.load(d + "/" + k + ".npy")).to(dev)
e, Y, V2, tau2, voff = ld("e"), ld("Y"), ld("V2"), ld("tau2"), ld("voff")
Yc = api.colmajor(Y.shape[0], Y.shape[1], torch.float64, dev)
Yc.copy_(Y)
n = Y.shape[0]
for rm in (True, False):
    Z = api.stage_bt2(e, Yc, 0, n, V2, tau2, voff, 64, rowmajor=rm)
    torch.cuda.synchronize()
    np.save(d + "/Z%d.npy" % int(rm), Z.cpu().numpy())
"""


def test_bt2_band64_pipelined_kernel_matches_ring(dev, tmp_path):
    """Band 64 has two back-transformation-2 kernels: the ring-window one (the
    default) and the pipelined one, selected by BDG_BT2_RING=0 (read once per
    process, hence the child process).  Both apply the same block reflectors
    in the same order; their outputs agree to rounding, on both Z routes."""
    import os
    import subprocess
    import sys
    import torch
    from paper_2310_03341_amd import api
    n, band = 301, 64
    ABh = random_band(n, band, seed=7)
    AB = torch.from_numpy(ABh).to(dev)
    d, e, V2, tau2, voff = api.stage_hb2st(AB, band)
    torch.cuda.synchronize()
    ea = torch.from_numpy(np.abs(e.cpu().numpy()[: n - 1]).copy()).to(dev)
    W, Y = api.stage_stedc(d, ea)
    torch.cuda.synchronize()
    for k, v in (("e", e), ("Y", Y), ("V2", V2), ("tau2", tau2), ("voff", voff)):
        np.save(str(tmp_path / (k + ".npy")), v.cpu().numpy())
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, BDG_BT2_RING="0")
    r = subprocess.run([sys.executable, "-c", _CHILD_BT2, str(tmp_path), root], env=env,
                       capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stderr[-2000:]
    for rm in (True, False):
        Zr = api.stage_bt2(e, Y, 0, n, V2, tau2, voff, band, rowmajor=rm)
        torch.cuda.synchronize()
        Zp = np.load(str(tmp_path / ("Z%d.npy" % int(rm))))
        assert np.abs(Zr.cpu().numpy() - Zp).max() < 1e-12, rm
