"""CPU oracle for the BdG eigenproblem -- TEST INFRASTRUCTURE ONLY.

Plain FP64 CPU implementations of what the GPU library computes, used to
check it.  Only the test-suite, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the product path never
does.  It shares no code with the GPU library: the only common module is the
seeded input generator (``paper_2310_03341_amd.inputs``), which holds none of
the method's arithmetic.

Contents
  * ``kinetic_1d``, ``assemble``: BdG matrix of eq. (stHpsi) on the spectral
    grid of "Numerical setup and implementation" (direct Fourier sum).
  * ``eigh_jacobi``: complex cyclic Jacobi (Golub & Van Loan sec. 8.5).
  * ``eigh_hqr``: Householder tridiagonalisation + implicit QL (G&VL sec. 8.3).
  * ``tridiag_eigh``, ``sturm_count``, ``bisect``: real tridiagonal helpers.
  * ``eigh``: dispatcher (Jacobi for small n, Householder+QL otherwise), with
    an optional closed energy window [emin, emax] as in the density sums of
    eq. (densities2).
  * ``assemble_entries``: selected entries of H from the same definition.
  * ``apply_h``: H applied to vectors without forming H (one 1-D kinetic
    matrix per lattice axis, then the local U - mu and Delta terms), for
    residuals of eigenvectors at sizes where the dense H does not fit the CPU.
Further oracle modules: ``oracle.scf`` (densities and SCF update),
``oracle.refine`` (Ogita-Aishima refinement step), ``oracle.net`` (conv net).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def build_mutant(k: int, out_dir: str) -> str:
    """Compile a copy with planted mistake k (for the pin self-test only)."""
    path = os.path.join(out_dir, "_oracle_mutant%d.so" % k)
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-D_GNU_SOURCE", "-DORACLE_MUTANT=%d" % k, "-o", path, _SRC, "-lm"])
    return path


def use_library(path):
    """Swap the loaded C library (None restores the default build)."""
    global _lib
    _lib = None
    _load(path)


def _load(path=None):
    global _lib
    if _lib is None:
        if path is None:
            build()
            path = _SO
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.oracle_kinetic_1d.argtypes = [ctypes.c_int, P, P]
        lib.oracle_assemble.argtypes = [ctypes.c_int, P, P, P, ctypes.c_double, P]
        lib.oracle_zheev_jacobi.argtypes = [ctypes.c_int, P, P, P, ctypes.c_double, ctypes.c_int]
        lib.oracle_zhetrd.argtypes = [ctypes.c_int, P, P, P, P]
        lib.oracle_zheev_hqr.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.oracle_dstev.argtypes = [ctypes.c_int, P, P, P, P]
        lib.oracle_sturm_count.argtypes = [ctypes.c_int64, P, P, ctypes.c_double]
        lib.oracle_sturm_count.restype = ctypes.c_int64
        lib.oracle_bisect.argtypes = [ctypes.c_int64, P, P, ctypes.c_int64]
        lib.oracle_bisect.restype = ctypes.c_double
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def kinetic_1d(N: int, return_imag: bool = False):
    """Kinetic matrix (1/N) sum_k (k^2/2) e^{ik(a-b)}, k = 2 pi n/N, n=-N/2..N/2-1."""
    T = np.zeros((N, N), order="F")
    Ti = np.zeros((N, N), order="F")
    _load().oracle_kinetic_1d(N, _p(T), _p(Ti))
    return (T, Ti) if return_imag else T


def assemble(dims, U, Delta, mu) -> np.ndarray:
    """Dense BdG matrix H (complex128, n x n, Fortran order) -- eq. (stHpsi)."""
    dims = [int(v) for v in dims]
    ns = int(np.prod(dims))
    U = np.ascontiguousarray(U, dtype=np.float64)
    D = np.ascontiguousarray(Delta, dtype=np.complex128)
    assert U.size == ns and D.size == ns
    H = np.zeros((2 * ns, 2 * ns), dtype=np.complex128, order="F")
    d = np.array(dims, dtype=np.int32)
    rc = _load().oracle_assemble(len(dims), _p(d), _p(U), _p(D), float(mu), _p(H))
    if rc != 0:
        raise ValueError("oracle_assemble failed (%d)" % rc)
    return H


def assemble_workload(w) -> np.ndarray:
    return assemble(w.dims, w.U, w.Delta, w.mu)


def eigh_jacobi(H: np.ndarray, tol: float = 2.2e-16, max_sweeps: int = 60):
    """Complex cyclic Jacobi: ascending W and orthonormal Z with H Z = Z W."""
    n = H.shape[0]
    A = np.array(H, dtype=np.complex128, order="F", copy=True)
    W = np.zeros(n)
    Z = np.zeros((n, n), dtype=np.complex128, order="F")
    sweeps = _load().oracle_zheev_jacobi(n, _p(A), _p(W), _p(Z), float(tol), int(max_sweeps))
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    return W, Z


def eigh_hqr(H: np.ndarray, vectors: bool = True, return_tridiag: bool = False):
    """Householder -> real tridiagonal -> implicit QL (+ back-transformation)."""
    n = H.shape[0]
    A = np.asfortranarray(H, dtype=np.complex128)
    W = np.zeros(n)
    Z = np.zeros((n, n), dtype=np.complex128, order="F") if vectors else None
    td = np.zeros(n)
    te = np.zeros(max(n - 1, 1))
    rc = _load().oracle_zheev_hqr(n, _p(A), _p(W), _p(Z) if vectors else None, _p(td), _p(te))
    if rc != 0:
        raise RuntimeError("QL did not converge")
    out = (W, Z)
    if return_tridiag:
        out = out + (td, te[: n - 1])
    return out


def tridiag_eigh(d, e, vectors: bool = True):
    """Eigenpairs of the real symmetric tridiagonal with diagonal d, off-diagonal e."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = d.size
    W = np.zeros(n)
    Y = np.zeros((n, n), order="F") if vectors else None
    ee = np.zeros(max(n, 1))
    ee[: n - 1] = e[: n - 1]
    rc = _load().oracle_dstev(n, _p(d), _p(ee), _p(W), _p(Y) if vectors else None)
    if rc != 0:
        raise RuntimeError("QL did not converge")
    return (W, Y) if vectors else W


def sturm_count(d, e, sigma: float) -> int:
    """Number of eigenvalues of the tridiagonal (d, e) strictly below sigma."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    return int(_load().oracle_sturm_count(d.size, _p(d), _p(e), float(sigma)))


def bisect(d, e, k: int) -> float:
    d = np.ascontiguousarray(d, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    return float(_load().oracle_bisect(d.size, _p(d), _p(e), int(k)))


def eigh(H: np.ndarray, emin: float = -np.inf, emax: float = np.inf, method: str = "auto"):
    """Eigenpairs of H with eigenvalues in the closed window [emin, emax]."""
    n = H.shape[0]
    if method == "auto":
        method = "jacobi" if n <= 256 else "hqr"
    W, Z = eigh_jacobi(H) if method == "jacobi" else eigh_hqr(H)
    sel = (W >= emin) & (W <= emax)
    return W[sel], Z[:, sel]


def assemble_entries(dims, U, Delta, mu, rows, cols) -> np.ndarray:
    """Selected entries H[rows[k], cols[k]] of the BdG matrix, from the same
    definition as ``assemble`` (direct Fourier sum for each axis), for sizes
    where the full matrix is too large for the CPU."""
    dims = [int(v) for v in dims]
    T = [kinetic_1d(N) for N in dims]
    ns = int(np.prod(dims))
    U = np.asarray(U, dtype=np.float64)
    D = np.asarray(Delta, dtype=np.complex128)

    def site(r):
        c = []
        for N in dims:
            c.append(r % N)
            r //= N
        return c

    out = np.zeros(len(rows), dtype=np.complex128)
    for k, (i, j) in enumerate(zip(rows, cols)):
        bi, bj = i >= ns, j >= ns
        si, sj = i - ns * bi, j - ns * bj
        if bi == bj:
            ci, cj = site(si), site(sj)
            h = 0.0
            for d in range(len(dims)):
                if all(ci[e] == cj[e] for e in range(len(dims)) if e != d):
                    h += T[d][ci[d], cj[d]]
            if si == sj:
                h += U[si] - mu
            out[k] = -h if bi else h
        elif si == sj:
            out[k] = np.conj(D[si]) if bi else D[si]
    return out


def apply_h(dims, U, Delta, mu, Z) -> np.ndarray:
    """H @ Z for the BdG matrix of eq. (stHpsi) without forming H.

    Z is (n, k) with rows [u; v], site index r = x + Nx (y + Ny z).  The
    kinetic operator of "Numerical setup and implementation" is separable:
    h acts on u as sum_d T_d along axis d (T_d from ``kinetic_1d``, the direct
    Fourier sum) plus the local U(r) - mu.  Then
        (H z)_u = h u + Delta v,     (H z)_v = conj(Delta) u - conj(h) v.
    """
    dims = [int(v) for v in dims]
    ns = int(np.prod(dims))
    Z = np.asarray(Z, dtype=np.complex128)
    if Z.ndim == 1:
        return apply_h(dims, U, Delta, mu, Z[:, None])[:, 0]
    k = Z.shape[1]
    assert Z.shape[0] == 2 * ns
    U = np.asarray(U, dtype=np.float64)
    D = np.asarray(Delta, dtype=np.complex128)
    # array axes (z, y, x, column) in C order put x fastest
    shape = tuple(reversed(dims)) + (k,)

    def kin(f, conj):
        f = f.reshape(shape)
        out = np.zeros(shape, dtype=np.complex128)
        for d, N in enumerate(dims):
            T = kinetic_1d(N)
            if conj:
                T = T.conj()
            ax = len(dims) - 1 - d
            out += np.moveaxis(np.tensordot(T, f, axes=([1], [ax])), 0, ax)
        return out.reshape(ns, k)

    u, v = Z[:ns], Z[ns:]
    loc = (U - mu)[:, None]
    hu = kin(u, False) + loc * u
    hv = kin(v, True) + loc * v
    return np.vstack([hu + D[:, None] * v, D.conj()[:, None] * u - hv])
