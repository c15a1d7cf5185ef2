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
