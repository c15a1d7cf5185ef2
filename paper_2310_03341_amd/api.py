"""Thin Python binding of libbdg.so: argument marshalling only.

Every computation runs in the HIP library; this module only passes device
pointers (from torch tensors), sizes and the current HIP stream across the
C-ABI declared in include/bdg.h.  If the library is not built, or there is no
GPU, the calls raise -- there is no CPU fallback.

Matrices are column-major.  A column-major n x n torch view is created as
``torch.empty((n, ld), dtype).T[:n]`` so that ``M[i, j]`` is element (i, j)
and ``M.stride(1)`` is the leading dimension.
"""
from __future__ import annotations

import ctypes
import math
import warnings
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbdg.so")
_lib = None

BDG_FP64 = 0
BDG_FP32_REFINED = 1


class BdgError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__("%s failed with status %d: %s" % (fn, code, msg))
        self.code = code


class Lattice(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dims", ctypes.c_int32 * 3)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("band", ctypes.c_int32),
                ("refine_max_iter", ctypes.c_int32), ("refine_tol", ctypes.c_double),
                ("dc_leaf", ctypes.c_int32), ("ph_mirror", ctypes.c_int32),
                ("max_pairs", ctypes.c_int64)]


class Report(ctypes.Structure):
    _fields_ = [("max_resid", ctypes.c_double), ("gram_defect", ctypes.c_double),
                ("eig_shift_max", ctypes.c_double), ("refine_iters", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("stage_ms", ctypes.c_double * 8),
                ("bt2_kernel_ms", ctypes.c_double), ("refine_close_pairs", ctypes.c_int32),
                ("refine_cluster_cols", ctypes.c_int32)]


def lib():
    """Load libbdg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libbdg.so is not built: run `python -m paper_2310_03341_amd.build` "
                               "(expected at %s)" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, I64, D, S = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        L.bdg_last_error.restype = ctypes.c_char_p
        L.bdg_version.restype = ctypes.c_char_p
        L.bdg_assemble.argtypes = [ctypes.POINTER(Lattice), P, P, D, P, I64, S]
        L.bdg_eigh_workspace.argtypes = [I64, ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_size_t)]
        L.bdg_eigh.argtypes = [I64, P, I64, D, D, P, P, I64, I64, ctypes.POINTER(I64),
                               ctypes.POINTER(Opts), P, ctypes.c_size_t, ctypes.POINTER(Report), S]
        L.bdg_check.argtypes = [I64, P, I64, I64, P, P, I64, ctypes.POINTER(D), ctypes.POINTER(D),
                                P, ctypes.c_size_t, S]
        L.bdg_zgemm.argtypes = [ctypes.c_char, ctypes.c_char, I64, I64, I64, P, P, I64, P, I64,
                                P, P, I64, S]
        L.bdg_cgemm.argtypes = L.bdg_zgemm.argtypes
        L.bdg_dgemm.argtypes = [ctypes.c_char, ctypes.c_char, I64, I64, I64, D, P, I64, P, I64,
                                D, P, I64, S]
        L.bdg_refine_workspace.argtypes = [I64, I64, ctypes.POINTER(ctypes.c_size_t)]
        L.bdg_refine.argtypes = [I64, P, I64, P, P, I64, I64, I64, P, ctypes.POINTER(Opts), P,
                                 ctypes.c_size_t, ctypes.POINTER(Report), S]
        _lib = L
    return _lib


BDG_ERR_REFINE_TOL = 2


def _call(name: str, *args, warn_codes=()) -> int:
    rc = getattr(lib(), name)(*args)
    if rc in warn_codes:
        warnings.warn("%s: %s" % (name, lib().bdg_last_error().decode()), RuntimeWarning, stacklevel=3)
    elif rc != 0:
        raise BdgError(name, rc, lib().bdg_last_error().decode())
    return rc


def _stream(dev=None) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _dev(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return t.data_ptr()


def colmajor(n: int, m: int, dtype, device="cuda", ld: Optional[int] = None) -> torch.Tensor:
    """Uninitialised column-major n x m tensor (M[i, j] = element (i, j))."""
    ld = ld or max(n, 1)
    return torch.empty((m, ld), dtype=dtype, device=device).T[:n]


def to_colmajor(M: torch.Tensor) -> torch.Tensor:
    out = colmajor(M.shape[0], M.shape[1], M.dtype, M.device)
    out.copy_(M)
    return out


def _ld(M: torch.Tensor) -> int:
    if M.dim() != 2 or M.stride(0) != 1:
        raise ValueError("expected a column-major matrix view (stride(0) == 1)")
    return max(M.stride(1), M.shape[0], 1)


def version() -> str:
    return lib().bdg_version().decode()


def assemble(dims: Sequence[int], U: torch.Tensor, Delta: torch.Tensor, mu: float,
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Dense BdG matrix (complex128, column-major) of eq. (stHpsi)."""
    lat = Lattice()
    lat.ndim = len(dims)
    for d, v in enumerate(dims):
        lat.dims[d] = int(v)
    n = 2 * int(math.prod(dims))
    H = out if out is not None else colmajor(n, n, torch.complex128, U.device)
    _call("bdg_assemble", ctypes.byref(lat), _dev(U), _dev(Delta), float(mu), _dev(H), _ld(H),
          _stream(U.device))
    return H


def make_opts(precision: int = BDG_FP64, band: int = 0, refine_max_iter: int = 0,
              refine_tol: float = 0.0, dc_leaf: int = 0, ph_mirror: int = 0,
              max_pairs: int = 0) -> Opts:
    o = Opts()
    o.precision, o.band, o.refine_max_iter = precision, band, refine_max_iter
    o.refine_tol, o.dc_leaf, o.ph_mirror = refine_tol, dc_leaf, ph_mirror
    o.max_pairs = max_pairs
    return o


def eigh_workspace(n: int, opts: Optional[Opts] = None) -> int:
    nb = ctypes.c_size_t(0)
    _call("bdg_eigh_workspace", int(n), ctypes.byref(opts) if opts else None, ctypes.byref(nb))
    return int(nb.value)


class Solver:
    """Holds the device workspace of bdg_eigh for one matrix order."""

    def __init__(self, n: int, opts: Optional[Opts] = None, device="cuda"):
        self.n = int(n)
        self.opts = opts or make_opts()
        self.bytes = eigh_workspace(self.n, self.opts)
        self.work = torch.empty(max(self.bytes, 1), dtype=torch.uint8, device=device)
        self.report = Report()

    def __call__(self, A: torch.Tensor, emin: float = -math.inf, emax: float = math.inf,
                 W: Optional[torch.Tensor] = None, Z: Optional[torch.Tensor] = None):
        n = self.n
        if A.shape != (n, n):
            raise ValueError("A must be %d x %d" % (n, n))
        W = W if W is not None else torch.empty(n, dtype=torch.float64, device=A.device)
        Z = Z if Z is not None else colmajor(n, n, torch.complex128, A.device)
        m = ctypes.c_int64(0)
        _call("bdg_eigh", n, _dev(A), _ld(A), float(emin), float(emax), _dev(W), _dev(Z),
              _ld(Z), Z.shape[1], ctypes.byref(m), ctypes.byref(self.opts), _dev(self.work),
              self.bytes, ctypes.byref(self.report), _stream(A.device),
              warn_codes=(BDG_ERR_REFINE_TOL,))
        k = int(m.value)
        return W[:k], Z[:, :k]


def eigh(A: torch.Tensor, emin: float = -math.inf, emax: float = math.inf,
         opts: Optional[Opts] = None):
    """Eigenpairs of the Hermitian A (destroyed) with eigenvalues in [emin, emax]."""
    return Solver(A.shape[0], opts, A.device)(A, emin, emax)


def gemm_int8(opA, opB, A, B, C, alpha=1.0, beta=0.0, slices: int = 8):
    """bdg_gemm_int8: C = alpha op(A) op(B) + beta C emulated in FP64 on the INT8
    matrix cores (float64 or complex128 column-major operands)."""
    L = lib()
    P, I64, S = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p
    L.bdg_gemm_int8_workspace.argtypes = [ctypes.c_int32, I64, I64, I64, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_size_t)]
    L.bdg_gemm_int8.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_char, ctypes.c_char, I64, I64, I64, P, P,
                                I64, P, I64, P, P, I64, P, ctypes.c_size_t, S]
    cplx = 1 if C.dtype == torch.complex128 else 0
    M, N = C.shape
    K = A.shape[0] if opA.upper() in ("C", "T") else A.shape[1]
    nb = ctypes.c_size_t(0)
    _call("bdg_gemm_int8_workspace", cplx, M, N, K, int(slices), ctypes.byref(nb))
    work = torch.empty(int(nb.value), dtype=torch.uint8, device=C.device)
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    _call("bdg_gemm_int8", cplx, int(slices), opA.encode(), opB.encode(), M, N, K,
          ctypes.cast(al, ctypes.c_void_p), _dev(A), _ld(A), _dev(B), _ld(B), ctypes.cast(be, ctypes.c_void_p),
          _dev(C), _ld(C), _dev(work), work.numel(), _stream(C.device))
    return C


def eigh1(A: torch.Tensor, emin: float = -math.inf, emax: float = math.inf, W=None, Z=None):
    """bdg_eigh1, the one-stage solver: real symmetric (float64 A) or complex
    Hermitian (complex128 A) column-major A, destroyed.  Returns (W, Z, report)."""
    L = lib()
    P, I64, D, S = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    L.bdg_eigh1_workspace.argtypes = [I64, ctypes.c_int32, I64, ctypes.POINTER(ctypes.c_size_t)]
    L.bdg_eigh1.argtypes = [I64, ctypes.c_int32, P, I64, D, D, P, P, I64, I64, ctypes.POINTER(I64), P,
                            ctypes.c_size_t, ctypes.POINTER(Report), S]
    n = A.shape[0]
    real = 1 if A.dtype == torch.float64 else 0
    if not real and A.dtype != torch.complex128:
        raise ValueError("A must be float64 (symmetric) or complex128 (Hermitian)")
    W = W if W is not None else torch.empty(n, dtype=torch.float64, device=A.device)
    Z = Z if Z is not None else colmajor(n, n, A.dtype, A.device)
    nb = ctypes.c_size_t(0)
    _call("bdg_eigh1_workspace", n, real, Z.shape[1], ctypes.byref(nb))
    work = torch.empty(int(nb.value), dtype=torch.uint8, device=A.device)
    rep = Report()
    m = ctypes.c_int64(0)
    _call("bdg_eigh1", n, real, _dev(A), _ld(A), float(emin), float(emax), _dev(W), _dev(Z), _ld(Z), Z.shape[1],
          ctypes.byref(m), _dev(work), work.numel(), ctypes.byref(rep), _stream(A.device))
    k = int(m.value)
    return W[:k], Z[:, :k], rep


def refine_workspace(n: int, m: int) -> int:
    nb = ctypes.c_size_t(0)
    _call("bdg_refine_workspace", int(n), int(m), ctypes.byref(nb))
    return int(nb.value)


def refine(H: torch.Tensor, lam: torch.Tensor, X: torch.Tensor, i0: int, m: int,
           opts: Optional[Opts] = None, W: Optional[torch.Tensor] = None):
    """FP64 refinement of columns [i0, i0 + m) of the approximate eigenbasis X
    (n x n complex128, column-major; refined in place) of the Hermitian H,
    lam the approximate eigenvalues of all n columns.  Returns (W, report):
    W[k] is the refined eigenvalue of column i0 + k."""
    n = H.shape[0]
    if X.shape != (n, n) or lam.numel() != n:
        raise ValueError("X must be n x n and lam hold n values")
    W = W if W is not None else torch.empty(max(m, 1), dtype=torch.float64, device=H.device)
    nb = refine_workspace(n, m)
    work = torch.empty(max(nb, 1), dtype=torch.uint8, device=H.device)
    rep = Report()
    _call("bdg_refine", n, _dev(H), _ld(H), _dev(lam), _dev(X), _ld(X), int(i0), int(m), _dev(W),
          ctypes.byref(opts) if opts is not None else None, _dev(work), nb, ctypes.byref(rep),
          _stream(H.device), warn_codes=(BDG_ERR_REFINE_TOL,))
    return W[:m], rep


def check(H: torch.Tensor, W: torch.Tensor, Z: torch.Tensor):
    """(max residual / ||H||_2, max |Z^H Z - I|) computed on the GPU in FP64."""
    n, m = Z.shape
    work = torch.empty(16 * (n * m + m * m) + 64, dtype=torch.uint8, device=H.device)
    r, g = ctypes.c_double(0), ctypes.c_double(0)
    _call("bdg_check", n, _dev(H), _ld(H), m, _dev(W), _dev(Z) if m else None, _ld(Z) if m else n,
          ctypes.byref(r), ctypes.byref(g), _dev(work), work.numel(), _stream(H.device))
    return r.value, g.value


def _gemm(fn: str, opA: str, opB: str, A, B, C, alpha, beta, real=False):
    M, N = C.shape
    K = A.shape[1] if opA == "N" else A.shape[0]
    if real:
        _call(fn, opA.encode(), opB.encode(), M, N, K, float(alpha), _dev(A), _ld(A), _dev(B),
              _ld(B), float(beta), _dev(C), _ld(C), _stream(C.device))
        return C
    ctype = ctypes.c_double if fn == "bdg_zgemm" else ctypes.c_float
    al = (ctype * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctype * 2)(complex(beta).real, complex(beta).imag)
    _call(fn, opA.encode(), opB.encode(), M, N, K, ctypes.cast(al, ctypes.c_void_p), _dev(A), _ld(A),
          _dev(B), _ld(B), ctypes.cast(be, ctypes.c_void_p), _dev(C), _ld(C), _stream(C.device))
    return C


def zgemm(opA, opB, A, B, C, alpha=1.0, beta=0.0):
    return _gemm("bdg_zgemm", opA, opB, A, B, C, alpha, beta)


def cgemm(opA, opB, A, B, C, alpha=1.0, beta=0.0):
    return _gemm("bdg_cgemm", opA, opB, A, B, C, alpha, beta)


def dgemm(opA, opB, A, B, C, alpha=1.0, beta=0.0):
    return _gemm("bdg_dgemm", opA, opB, A, B, C, alpha, beta, real=True)


# ---------------------------------------------------------------- stage hooks
def _stage_sigs(L):
    P, I64, S = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p
    L.bdg_stage_workspace.argtypes = [ctypes.c_int, I64, ctypes.c_int, I64,
                                      ctypes.POINTER(ctypes.c_size_t)]
    L.bdg_stage_nrefl.argtypes = [I64, ctypes.c_int]
    L.bdg_stage_nrefl.restype = I64
    L.bdg_stage_he2hb.argtypes = [I64, P, I64, ctypes.c_int, P, I64, P, P, ctypes.c_size_t, S]
    L.bdg_stage_hb2st.argtypes = [I64, ctypes.c_int, P, I64, P, P, P, P, P, S]
    L.bdg_stage_stedc.argtypes = [I64, P, P, P, P, ctypes.c_int, P, ctypes.c_size_t, S]
    L.bdg_stage_bt2.argtypes = [I64, ctypes.c_int, I64, P, P, I64, P, P, P, P, I64, P,
                                ctypes.c_size_t, S]
    L.bdg_stage_bt1.argtypes = [I64, I64, P, I64, ctypes.c_int, P, P, I64, P, ctypes.c_size_t, S]


def stage_workspace(stage: int, n: int, band: int = 64, m: int = 0, device="cuda"):
    L = lib()
    _stage_sigs(L)
    nb = ctypes.c_size_t(0)
    _call("bdg_stage_workspace", stage, n, band, m, ctypes.byref(nb))
    return torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=device)


def stage_he2hb(A: torch.Tensor, band: int = 64):
    """Stage 1 on A (destroyed): returns (AB, T1) device tensors."""
    L = lib()
    _stage_sigs(L)
    n = A.shape[0]
    ldab = 2 * band + 2
    AB = torch.zeros((n, ldab), dtype=torch.complex128, device=A.device)  # AB[j, d]
    np_ = max(1, sum(1 for k in range(0, n, band) if k + band + 1 < n))
    T1 = torch.zeros(np_ * band * band, dtype=torch.complex128, device=A.device)
    work = stage_workspace(1, n, band, 0, A.device)
    _call("bdg_stage_he2hb", n, _dev(A), _ld(A), band, _dev(AB), ldab, _dev(T1), _dev(work),
          work.numel(), _stream(A.device))
    return AB, T1


def stage_hb2st(AB: torch.Tensor, band: int = 64):
    """Stage 2 on AB (destroyed): returns (d, e_complex, V2, tau2, voff)."""
    L = lib()
    _stage_sigs(L)
    n, ldab = AB.shape
    nrefl = int(L.bdg_stage_nrefl(n, band))
    dev = AB.device
    d = torch.zeros(n, dtype=torch.float64, device=dev)
    e = torch.zeros(max(n, 1), dtype=torch.complex128, device=dev)
    V2 = torch.zeros((nrefl + 1) * band, dtype=torch.complex128, device=dev)
    tau2 = torch.zeros(nrefl + 1, dtype=torch.float64, device=dev)
    voff = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    _call("bdg_stage_hb2st", n, band, _dev(AB), ldab, _dev(d), _dev(e), _dev(V2), _dev(tau2),
          _dev(voff), _stream(dev))
    return d, e, V2, tau2, voff


def stage_stedc(d: torch.Tensor, e: torch.Tensor, leaf: int = 0):
    L = lib()
    _stage_sigs(L)
    n = d.numel()
    W = torch.zeros(n, dtype=torch.float64, device=d.device)
    Q = colmajor(n, n, torch.float64, d.device)
    work = stage_workspace(3, n, 64, 0, d.device)
    ee = e if e.numel() > 0 else torch.zeros(1, dtype=torch.float64, device=d.device)
    _call("bdg_stage_stedc", n, _dev(d), _dev(ee), _dev(W), _dev(Q), leaf, _dev(work),
          work.numel(), _stream(d.device))
    return W, Q


def stage_bt2(e_cplx, Y, i0, m, V2, tau2, voff, band: int = 64, rowmajor: bool = True):
    """rowmajor=False passes a workspace without room for the row-major copy
    of Z, which makes the library take its column-major route."""
    L = lib()
    _stage_sigs(L)
    n = Y.shape[0]
    Z = colmajor(n, max(m, 1), torch.complex128, Y.device)
    work = stage_workspace(4, n, band, m, Y.device)
    nbytes = work.numel()
    if not rowmajor and band % 16 == 0:
        nbytes -= 16 * n * max(m, 0)
    _call("bdg_stage_bt2", n, band, m, _dev(e_cplx), _dev(Y), i0, _dev(V2), _dev(tau2), _dev(voff),
          _dev(Z), _ld(Z), _dev(work), nbytes, _stream(Y.device))
    return Z[:, :m]


def stage_zgemm(mode: int, splitk: int, opA: str, opB: str, A, B, C, alpha=1.0, beta=0.0):
    """The complex128 tile GEMM in mode 0 (full), 1 (lower tiles) or 2 (Hermitian
    A from its lower triangle) with K split into `splitk` chunks."""
    L = lib()
    P, I64, S = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p
    L.bdg_stage_zgemm.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_char, ctypes.c_char, I64, I64,
                                  I64, P, P, I64, P, I64, P, P, I64, P, ctypes.c_size_t, S]
    M, N = C.shape
    K = A.shape[1] if opA == "N" else A.shape[0]
    nb = 16 * splitk * M * N if splitk > 1 else 0
    work = torch.empty(max(nb, 1), dtype=torch.uint8, device=C.device)
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    _call("bdg_stage_zgemm", mode, splitk, opA.encode(), opB.encode(), M, N, K,
          ctypes.cast(al, ctypes.c_void_p), _dev(A), _ld(A), _dev(B), _ld(B),
          ctypes.cast(be, ctypes.c_void_p), _dev(C), _ld(C), _dev(work), nb, _stream(C.device))
    return C


def stage_bt1(A, T1, Z, band: int = 64):
    L = lib()
    _stage_sigs(L)
    n, m = Z.shape
    work = stage_workspace(5, n, band, m, Z.device)
    _call("bdg_stage_bt1", n, m, _dev(A), _ld(A), band, _dev(T1), _dev(Z), _ld(Z), _dev(work),
          work.numel(), _stream(Z.device))
    return Z


# ---------------------------------------------------------------- SCF step
class ScfParamsC(ctypes.Structure):
    _fields_ = [("B", ctypes.c_double), ("g", ctypes.c_double), ("alpha", ctypes.c_double),
                ("Ec", ctypes.c_double), ("T", ctypes.c_double), ("regularize", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


def _scf_sigs(L):
    P, I64, D, S = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    L.bdg_scf_workspace.argtypes = [ctypes.POINTER(Lattice), ctypes.POINTER(ctypes.c_size_t)]
    L.bdg_scf_step.argtypes = [ctypes.POINTER(Lattice), P, P, D, ctypes.POINTER(ScfParamsC), P, P, P,
                               P, ctypes.POINTER(D), ctypes.POINTER(I64), P, ctypes.c_size_t, S]
    L.bdg_regrid.argtypes = [ctypes.POINTER(Lattice), P, ctypes.POINTER(Lattice), P, D, S]


def regrid(src_dims, f: torch.Tensor, dst_dims, scale: float = 1.0) -> torch.Tensor:
    """bdg_regrid: the field f on lattice src_dims moved to dst_dims (trigonometric
    interpolation to a finer lattice, injection to a coarser one), times scale."""
    L = lib()
    _scf_sigs(L)
    src, dst = Lattice(), Lattice()
    for lat, dims in ((src, src_dims), (dst, dst_dims)):
        lat.ndim = len(dims)
        for d, v in enumerate(dims):
            lat.dims[d] = int(v)
    g = torch.empty(math.prod(int(v) for v in dst_dims), dtype=torch.float64, device=f.device)
    _call("bdg_regrid", ctypes.byref(src), _dev(f), ctypes.byref(dst), _dev(g), float(scale), _stream(f.device))
    return g


class TdParamsC(ctypes.Structure):
    _fields_ = [("B", ctypes.c_double), ("g", ctypes.c_double), ("self_consistent", ctypes.c_int32),
                ("resume", ctypes.c_int32)]


class TdEvolver:
    """Workspace (and so the integrator's history) of bdg_td_evolve for m states
    on one lattice.  evolve() advances Phi [n x m] (column-major, complex128) in
    place; the first call starts fresh, later calls continue the history."""

    def __init__(self, dims, m: int, mu: float, B: float = 0.0, g: float = 0.0, Vext=None, U0=None, D0=None,
                 self_consistent: bool = True, device="cuda"):
        L = lib()
        P, I64, D, S = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        L.bdg_td_workspace.argtypes = [ctypes.POINTER(Lattice), I64, ctypes.POINTER(ctypes.c_size_t)]
        L.bdg_td_evolve.argtypes = [ctypes.POINTER(Lattice), P, D, ctypes.POINTER(TdParamsC), I64, P, I64, D, I64,
                                    P, P, P, ctypes.c_size_t, S]
        self.lat = Lattice()
        self.lat.ndim = len(dims)
        for d, v in enumerate(dims):
            self.lat.dims[d] = int(v)
        self.m, self.mu = int(m), float(mu)
        self.p = TdParamsC(float(B), float(g), int(bool(self_consistent)), 0)
        self.Vext, self.U0, self.D0 = Vext, U0, D0
        nb = ctypes.c_size_t(0)
        _call("bdg_td_workspace", ctypes.byref(self.lat), self.m, ctypes.byref(nb))
        self.work = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        self.started = False

    def evolve(self, Phi: torch.Tensor, dt: float, nsteps: int):
        self.p.resume = 1 if self.started else 0
        opt = lambda t: _dev(t) if t is not None else None  # noqa: E731
        _call("bdg_td_evolve", ctypes.byref(self.lat), opt(self.Vext), self.mu, ctypes.byref(self.p), self.m,
              _dev(Phi), _ld(Phi), float(dt), int(nsteps), opt(self.U0), opt(self.D0), _dev(self.work),
              self.work.numel(), _stream(Phi.device))
        self.started = True
        return Phi


class ScfStepper:
    """Workspace + fixed inputs of the SCF step on one lattice (device tensors)."""

    def __init__(self, dims, Vext: torch.Tensor, theta: torch.Tensor, mu: float, params):
        L = lib()
        _scf_sigs(L)
        self.lat = Lattice()
        self.lat.ndim = len(dims)
        for d, v in enumerate(dims):
            self.lat.dims[d] = int(v)
        self.Vext, self.theta, self.mu = Vext, theta, float(mu)
        self.p = ScfParamsC(params.B, params.g, params.alpha, params.Ec, float(getattr(params, "T", 0.0)),
                            int(getattr(params, "regularize", 0)), 0)
        nb = ctypes.c_size_t(0)
        _call("bdg_scf_workspace", ctypes.byref(self.lat), ctypes.byref(nb))
        self.work = torch.empty(int(nb.value), dtype=torch.uint8, device=Vext.device)
        ns = Vext.numel()
        self.density = torch.zeros(ns, dtype=torch.float64, device=Vext.device)
        self.nu_abs = torch.zeros(ns, dtype=torch.float64, device=Vext.device)

    def step(self, U: torch.Tensor, absDelta: torch.Tensor):
        """In-place update of U and absDelta; returns (change, m)."""
        ch = ctypes.c_double(0.0)
        m = ctypes.c_int64(0)
        _call("bdg_scf_step", ctypes.byref(self.lat), _dev(self.Vext), _dev(self.theta), self.mu,
              ctypes.byref(self.p), _dev(U), _dev(absDelta), _dev(self.density), _dev(self.nu_abs),
              ctypes.byref(ch), ctypes.byref(m), _dev(self.work), self.work.numel(),
              _stream(U.device))
        return ch.value, int(m.value)


# ---------------------------------------------------------------- start-field network
class NetShape(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int32), ("ny", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("batch", ctypes.c_int32)]


def _net_sigs(L):
    P, I64, D, S = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    SH = ctypes.POINTER(NetShape)
    L.bdg_net_nparams.argtypes = [SH]
    L.bdg_net_nparams.restype = I64
    L.bdg_net_workspace.argtypes = [SH, ctypes.POINTER(ctypes.c_size_t)]
    L.bdg_net_forward.argtypes = [SH, P, P, P, D, P, P, ctypes.c_size_t, S]
    L.bdg_net_forward_noalloc.argtypes = [SH, P, P, P, D, P, S]
    L.bdg_net_backward.argtypes = [SH, P, P, P, D, P, P, P, P, ctypes.c_size_t, S]
    L.bdg_net_adam_step.argtypes = [I64, P, P, P, P, ctypes.c_int32, ctypes.c_float, S]
    L.bdg_net_start_fields.argtypes = [SH, P, ctypes.c_int32, P, P, P, S]


class StartNet:
    """Device state of the start-field network: FP32 master weights, Adam moments."""

    def __init__(self, channels: int, ny: int, nx: int, batch: int, device="cuda"):
        L = lib()
        _net_sigs(L)
        self.shape = NetShape(channels, ny, nx, batch)
        self.nparams = int(L.bdg_net_nparams(ctypes.byref(self.shape)))
        if self.nparams < 0:
            raise BdgError("bdg_net_nparams", -1, L.bdg_last_error().decode())
        nb = ctypes.c_size_t(0)
        _call("bdg_net_workspace", ctypes.byref(self.shape), ctypes.byref(nb))
        self.work = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        self.params = torch.zeros(self.nparams, dtype=torch.float32, device=device)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.t = 0
        self.device = device

    def forward(self, Vext: torch.Tensor, theta: torch.Tensor, mu: float, y=None):
        B = self.shape.batch
        P = self.shape.ny * self.shape.nx
        y = y if y is not None else torch.empty((B, 2, P), dtype=torch.float32, device=self.device)
        _call("bdg_net_forward", ctypes.byref(self.shape), _dev(self.params), _dev(Vext), _dev(theta),
              float(mu), _dev(y), _dev(self.work), self.work.numel(), _stream(self.device))
        return y

    def forward_noalloc(self, Vext: torch.Tensor, theta: torch.Tensor, mu: float, y: torch.Tensor):
        """bdg_net_forward_noalloc: the forward pass on the library's own device
        scratch (no workspace); y [batch, 2, ny*nx] FP32 is caller-allocated."""
        _call("bdg_net_forward_noalloc", ctypes.byref(self.shape), _dev(self.params), _dev(Vext), _dev(theta),
              float(mu), _dev(y), _stream(self.device))
        return y

    def start_fields(self, y: torch.Tensor, sample: int, Vext: torch.Tensor):
        """bdg_net_start_fields: (U, |Delta|) of output sample `sample` of y."""
        U = torch.empty_like(Vext)
        D = torch.empty_like(Vext)
        _call("bdg_net_start_fields", ctypes.byref(self.shape), _dev(y), int(sample), _dev(Vext), _dev(U), _dev(D),
              _stream(self.device))
        return U, D

    def backward(self, Vext, theta, mu, target):
        _call("bdg_net_backward", ctypes.byref(self.shape), _dev(self.params), _dev(Vext), _dev(theta),
              float(mu), _dev(target), _dev(self.grads), _dev(self.loss), _dev(self.work),
              self.work.numel(), _stream(self.device))
        return self.loss

    def adam(self, lr: float = 1e-3):
        self.t += 1
        _call("bdg_net_adam_step", self.nparams, _dev(self.params), _dev(self.grads), _dev(self.m),
              _dev(self.v), self.t, float(lr), _stream(self.device))
