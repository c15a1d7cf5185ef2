"""Planted mistakes in the oracle must fail at least one of its pins.

Each mutant is the oracle compiled with one plausible error (uncentred
momenta, wrong sign of the hole block, dropped mu, unconjugated pairing block,
a dropped Householder term, a wrong rotation sign, a transposed Jacobi phase,
an off-by-one Sturm recurrence).  The pins below are the same kinds of checks
as in test_oracle.py; the test passes when every mutant is caught.
"""
import numpy as np
import pytest
import scipy.linalg

from paper_2310_03341_amd import inputs
from tests.test_oracle import kinetic_closed_form, uniform_spectrum


def _pins(orc):
    """Run the pins; return the names of those that fail."""
    failed = []

    def check(name, fn):
        try:
            ok = fn()
        except Exception:
            ok = False
        if not ok:
            failed.append(name)

    check("kinetic", lambda: np.abs(orc.kinetic_1d(8) - kinetic_closed_form(8)).max() < 1e-12)
    w = inputs.line_3d_small((4, 4, 2))
    H = orc.assemble_workload(w)
    check("hermitian", lambda: np.abs(H - H.conj().T).max() < 1e-14)
    u = inputs.uniform((4, 4, 2), 0.1, 0.3 + 0.1j, 0.7)
    Hu = orc.assemble_workload(u)
    ref_u = uniform_spectrum(u.dims, 0.1, 0.3 + 0.1j, 0.7)
    check("uniform", lambda: np.abs(orc.eigh_hqr(Hu, vectors=False)[0] - ref_u).max() < 1e-12)
    R = inputs.random_hermitian(40, seed=5)
    ref = scipy.linalg.eigvalsh(R)

    def hqr_ok():
        W, Z = orc.eigh_hqr(R)
        return (np.abs(W - ref).max() < 1e-12 and np.abs(R @ Z - Z * W).max() < 1e-12)

    def jac_ok():
        W, Z = orc.eigh_jacobi(R)
        return (np.abs(W - ref).max() < 1e-12 and np.abs(R @ Z - Z * W).max() < 1e-12)

    check("hqr", hqr_ok)
    check("jacobi", jac_ok)
    d = np.full(50, 2.0)
    e = np.ones(49)
    ev = 2.0 - 2.0 * np.cos(np.arange(1, 51) * np.pi / 51)
    check("sturm", lambda: all(orc.sturm_count(d, e, s) == int(np.sum(ev < s))
                                for s in (0.5, 1.7, 3.2)))
    return failed


def test_default_build_passes_all_pins(orc):
    assert _pins(orc) == []


@pytest.mark.parametrize("k", range(1, 9))
def test_mutant_is_caught(orc, k, tmp_path):
    path = orc.build_mutant(k, str(tmp_path))
    orc.use_library(path)
    try:
        failed = _pins(orc)
    finally:
        orc.use_library(None)
    assert failed, "mutant %d passed every pin" % k
