"""Checkpoints of the self-consistent iteration (host-side files).

A checkpoint holds the fields U and |Delta| after a completed iteration, the
iteration count, the history of the update norms and a fingerprint of the
problem (lattice, chemical potential, functional and mixing parameters, and a
digest of V_ext and theta).  The SCF step is a function of the fields alone,
so continuing from a checkpoint reproduces the iteration that was
interrupted.  Files are numpy .npz archives of plain arrays (no pickled
objects) and are replaced atomically (write to a temporary name, then
rename), so an interruption during a write leaves the previous checkpoint.
"""
from __future__ import annotations

import hashlib
import os
from typing import Optional, Tuple

import numpy as np


def fingerprint(dims, mu: float, params, Vext: np.ndarray, theta: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.asarray(dims, dtype=np.int64).tobytes())
    fields = (float(mu), float(params.B), float(params.g), float(params.alpha), float(params.Ec),
              float(getattr(params, "T", 0.0)), float(getattr(params, "regularize", 0)))
    h.update(np.asarray(fields, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(Vext, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(theta, dtype=np.float64).tobytes())
    return h.hexdigest()


def save(path: str, U: np.ndarray, D: np.ndarray, it: int, hist, fp: str) -> None:
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "wb") as f:
        np.savez(f, U=np.asarray(U, dtype=np.float64), D=np.asarray(D, dtype=np.float64),
                 it=np.int64(it), hist=np.asarray(hist, dtype=np.float64),
                 fp=np.frombuffer(fp.encode("ascii"), dtype=np.uint8))
    os.replace(tmp, path)


def load(path: str, fp: str) -> Optional[Tuple[np.ndarray, np.ndarray, int, list]]:
    """The checkpoint at `path` if it exists; ValueError if it belongs to
    another problem (fingerprint mismatch)."""
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        got = bytes(z["fp"]).decode("ascii")
        if got != fp:
            raise ValueError("checkpoint %s belongs to another problem" % path)
        return z["U"].copy(), z["D"].copy(), int(z["it"]), [float(x) for x in z["hist"]]
