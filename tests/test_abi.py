"""The C-ABI library loads and exports every entry point that include/*.h declares."""
import glob
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    syms = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(bdg_[a-z0-9_]+)\s*\(", src):
            syms.add(m.group(1))
    return sorted(syms)


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("bdg_assemble", "bdg_eigh", "bdg_eigh_workspace", "bdg_check", "bdg_last_error"):
        assert s in syms


def test_library_exports_declared_symbols():
    from paper_2310_03341_amd import api
    if not os.path.exists(api.LIB_PATH):
        pytest.skip("libbdg.so not built")
    L = ctypes.CDLL(api.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing
    assert b"gfx950" in api.lib().bdg_version()


def test_argument_errors_without_gpu():
    """Host-side argument checks return LAPACK-style negative codes."""
    from paper_2310_03341_amd import api
    if not os.path.exists(api.LIB_PATH):
        pytest.skip("libbdg.so not built")
    L = api.lib()
    lat = api.Lattice()
    lat.ndim = 4
    assert L.bdg_assemble(ctypes.byref(lat), None, None, 0.0, None, 0, None) == -1
    lat.ndim = 2
    lat.dims[0], lat.dims[1] = 5, 4
    assert L.bdg_assemble(ctypes.byref(lat), None, None, 0.0, None, 0, None) == -1
    assert b"even" in L.bdg_last_error()
    nb = ctypes.c_size_t(0)
    assert L.bdg_eigh_workspace(0, None, ctypes.byref(nb)) == -1


def test_refine_argument_errors_without_gpu():
    from paper_2310_03341_amd import api
    if not os.path.exists(api.LIB_PATH):
        pytest.skip("libbdg.so not built")
    L = api.lib()
    P = ctypes.c_void_p(256)  # never dereferenced: every call below fails its argument check
    nb = ctypes.c_size_t(0)
    assert L.bdg_refine_workspace(10, 11, ctypes.byref(nb)) == -2
    assert L.bdg_refine_workspace(10, 4, ctypes.byref(nb)) == 0 and nb.value >= 2 * 16 * 10 * 4
    args = lambda **k: dict(dict(n=10, H=P, ldh=10, lam=P, X=P, ldx=10, i0=0, m=4, W=P), **k)  # noqa: E731

    def call(a):
        return L.bdg_refine(a["n"], a["H"], a["ldh"], a["lam"], a["X"], a["ldx"], a["i0"], a["m"],
                            a["W"], None, None, 0, None, None)
    assert call(args(n=0)) == -1
    assert call(args(H=None)) == -2
    assert call(args(ldh=9)) == -3
    assert call(args(lam=None)) == -4
    assert call(args(X=None)) == -5
    assert call(args(ldx=9)) == -6
    assert call(args(i0=-1)) == -7
    assert call(args(i0=8, m=3)) == -8
    assert call(args(W=None)) == -9
    assert call(args()) == 4  # no workspace: BDG_ERR_WORKSPACE
    o = api.make_opts(refine_max_iter=-1)
    assert L.bdg_refine(10, P, 10, P, P, 10, 0, 4, P, ctypes.byref(o), None, 0, None, None) == -10


def test_mixed_workspace_fits_largest_window():
    """The 32^3 ring (n = 65536) with the window [0, 6] (about 25,000 pairs):
    workspace of the mixed arm sized by max_pairs, plus H and a Z of 26,214
    columns, stays inside one MI355X's 288 GB (with 8 GB to spare)."""
    from paper_2310_03341_amd import api
    if not os.path.exists(api.LIB_PATH):
        pytest.skip("libbdg.so not built")
    n, zc = 65536, 26214
    nb = ctypes.c_size_t(0)
    o = api.make_opts(precision=api.BDG_FP32_REFINED, ph_mirror=1, max_pairs=zc)
    assert api.lib().bdg_eigh_workspace(n, ctypes.byref(o), ctypes.byref(nb)) == 0
    total = nb.value + 16 * n * n + 16 * n * zc
    assert total <= 280e9, total / 1e9
    full = api.make_opts(precision=api.BDG_FP32_REFINED, ph_mirror=1)
    assert api.lib().bdg_eigh_workspace(n, ctypes.byref(full), ctypes.byref(nb)) == 0
    assert nb.value > total - 16 * n * n - 16 * n * zc


def test_extension_argument_errors_without_gpu():
    """Host-side checks of the one-stage solver, the TDSLDA evolution, the
    regrid, the INT8 products and the network decode (no device call)."""
    from paper_2310_03341_amd import api
    if not os.path.exists(api.LIB_PATH):
        pytest.skip("libbdg.so not built")
    L = api.lib()
    I64, P, D = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
    nb = ctypes.c_size_t(0)
    L.bdg_eigh1_workspace.argtypes = [I64, ctypes.c_int32, I64, ctypes.POINTER(ctypes.c_size_t)]
    assert L.bdg_eigh1_workspace(0, 0, 1, ctypes.byref(nb)) == -1
    assert L.bdg_eigh1_workspace(10, 2, 1, ctypes.byref(nb)) == -2
    assert L.bdg_eigh1_workspace(10, 1, 10, ctypes.byref(nb)) == 0 and nb.value > 8 * 100
    L.bdg_eigh1.argtypes = [I64, ctypes.c_int32, P, I64, D, D, P, P, I64, I64, P, P, ctypes.c_size_t, P, P]
    X = ctypes.c_void_p(256)  # never dereferenced
    m = ctypes.c_int64(0)
    assert L.bdg_eigh1(10, 0, X, 5, 0.0, 1.0, X, X, 10, 10, ctypes.byref(m), X, 1 << 30, None, None) == -4
    assert L.bdg_eigh1(10, 0, X, 10, 2.0, 1.0, X, X, 10, 10, ctypes.byref(m), X, 1 << 30, None, None) == -5
    assert L.bdg_eigh1(10, 0, X, 10, 0.0, 1.0, X, X, 10, 10, ctypes.byref(m), X, 16, None, None) == 4
    # TDSLDA: more than 4096 sites is refused before any launch; bad dt
    lat = api.Lattice()
    lat.ndim = 3
    lat.dims[0], lat.dims[1], lat.dims[2] = 16, 16, 18
    prm = api.TdParamsC(0.0, 0.0, 1, 0)
    L.bdg_td_evolve.argtypes = [ctypes.POINTER(api.Lattice), P, D, ctypes.POINTER(api.TdParamsC), I64, P, I64, D,
                                I64, P, P, P, ctypes.c_size_t, P]
    assert L.bdg_td_evolve(ctypes.byref(lat), X, 1.0, ctypes.byref(prm), 2, X, 9216, 0.01, 1, None, None, X,
                           1 << 40, None) == 5
    lat.dims[2] = 8
    assert L.bdg_td_evolve(ctypes.byref(lat), X, 1.0, ctypes.byref(prm), 2, X, 4096, -0.01, 1, None, None, X,
                           1 << 40, None) == -8
    prm.self_consistent = 0
    assert L.bdg_td_evolve(ctypes.byref(lat), X, 1.0, ctypes.byref(prm), 2, X, 4096, 0.01, 1, None, None, X,
                           1 << 40, None) == -10
    # regrid: a target neither finer nor an integer coarsening
    a, b = api.Lattice(), api.Lattice()
    a.ndim = b.ndim = 2
    a.dims[0], a.dims[1], b.dims[0], b.dims[1] = 12, 12, 8, 14
    L.bdg_regrid.argtypes = [ctypes.POINTER(api.Lattice), P, ctypes.POINTER(api.Lattice), P, D, P]
    assert L.bdg_regrid(ctypes.byref(a), X, ctypes.byref(b), X, 1.0, None) == -3
    # INT8 products: slices outside 3..8, 'T' for complex
    L.bdg_gemm_int8.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_char, ctypes.c_char, I64, I64, I64, P, P,
                                I64, P, I64, P, P, I64, P, ctypes.c_size_t, P]
    one = (D * 2)(1.0, 0.0)
    assert L.bdg_gemm_int8(1, 2, b"N", b"N", 4, 4, 4, one, X, 4, X, 4, one, X, 4, X, 1 << 30, None) == -2
    assert L.bdg_gemm_int8(1, 8, b"T", b"N", 4, 4, 4, one, X, 4, X, 4, one, X, 4, X, 1 << 30, None) < 0
    # network decode: sample out of range
    sh = api.NetShape(8, 8, 8, 2)
    L.bdg_net_start_fields.argtypes = [ctypes.POINTER(api.NetShape), P, ctypes.c_int32, P, P, P, P]
    assert L.bdg_net_start_fields(ctypes.byref(sh), X, 2, X, X, X, None) == -3
