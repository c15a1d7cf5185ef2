"""SCF checkpoints on the host: an interrupted iteration continued from its
checkpoint gives the same iterates and history as an uninterrupted one, a
checkpoint of another problem is refused, and a finished run is not iterated
again.  The stepper here is a deterministic contraction on CPU tensors with
the SCF step's interface (in-place update, returns the update norm)."""
import math
import os

import numpy as np
import pytest
import torch

from paper_2310_03341_amd import checkpoint as ckpt
from paper_2310_03341_amd import inputs
from paper_2310_03341_amd.learned_start import run_scf


class Contraction:
    def __init__(self, n, seed=0):
        g = np.random.default_rng(seed)
        self.a = torch.from_numpy(g.standard_normal(n))
        self.b = torch.from_numpy(g.standard_normal(n))
        self.calls = 0

    def step(self, U, D):
        self.calls += 1
        U1 = 0.7 * U + 0.3 * torch.tanh(self.a + 0.5 * D)
        D1 = 0.6 * D + 0.4 * torch.cos(self.b + 0.5 * U)
        ch = float(torch.sqrt(((U1 - U) ** 2).sum() + ((D1 - D) ** 2).sum()))
        U.copy_(U1)
        D.copy_(D1)
        return ch, 0


def _params(tol, max_iter):
    return inputs.ScfParams(tol=tol, max_iter=max_iter)


def _start(n):
    return torch.zeros(n, dtype=torch.float64), torch.full((n,), 0.3, dtype=torch.float64)


def test_resume_reproduces_the_uninterrupted_iteration(tmp_path):
    n, tol = 50, 1e-12
    U, D = _start(n)
    it_a, ok_a, hist_a = run_scf(Contraction(n), U, D, _params(tol, 200))
    assert ok_a
    path = str(tmp_path / "scf.npz")
    fp = "problem-1"
    U2, D2 = _start(n)
    it_b, ok_b, _ = run_scf(Contraction(n), U2, D2, _params(tol, 13), checkpoint=path, every=5, fp=fp)
    assert not ok_b and it_b == 13 and os.path.exists(path)
    U3, D3 = torch.zeros(n, dtype=torch.float64), torch.zeros(n, dtype=torch.float64)
    st = Contraction(n)
    it_c, ok_c, hist_c = run_scf(st, U3, D3, _params(tol, 200), checkpoint=path, every=5, fp=fp)
    assert ok_c and it_c == it_a
    assert st.calls == it_a - 13
    assert hist_c == hist_a
    assert torch.equal(U3, U) and torch.equal(D3, D)
    # a finished run is read back without another step
    st2 = Contraction(n)
    U4, D4 = _start(n)
    it_d, ok_d, _ = run_scf(st2, U4, D4, _params(tol, 200), checkpoint=path, fp=fp)
    assert ok_d and it_d == it_a and st2.calls == 0 and torch.equal(U4, U)


def test_checkpoint_of_another_problem_is_refused(tmp_path):
    path = str(tmp_path / "scf.npz")
    ckpt.save(path, np.zeros(4), np.zeros(4), 3, [1.0, 0.5, 0.25], "a")
    with pytest.raises(ValueError):
        ckpt.load(path, "b")
    U, D, it, hist = ckpt.load(path, "a")
    assert it == 3 and hist == [1.0, 0.5, 0.25]


def test_fingerprint_separates_problems():
    p = inputs.ScfParams()
    V = np.linspace(0, 1, 16)
    th = np.zeros(16)
    a = ckpt.fingerprint((4, 4), 1.0, p, V, th)
    assert a == ckpt.fingerprint((4, 4), 1.0, p, V.copy(), th)
    assert a != ckpt.fingerprint((4, 4), 1.0 + 1e-15 * 4, p, V, th)
    V2 = V.copy()
    V2[3] += 1e-9
    assert a != ckpt.fingerprint((4, 4), 1.0, p, V2, th)
    assert a != ckpt.fingerprint((2, 8), 1.0, p, V, th)


def test_diverged_history_is_kept():
    class Bad(Contraction):
        def step(self, U, D):
            self.calls += 1
            return math.nan, 0
    U, D = _start(4)
    it, ok, hist = run_scf(Bad(4), U, D, _params(1e-9, 10))
    assert it == 1 and not ok and math.isnan(hist[0])


def test_bench_results_log_appends_json_lines(tmp_path):
    import importlib.util
    import json
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    path = str(tmp_path / "runs.jsonl")
    b.append_log(path, {"metric": "m", "value": 1.5})
    b.append_log(path, {"metric": "m", "value": 2.5})
    b.append_log("", {"ignored": True})
    rows = [json.loads(line) for line in open(path)]
    assert [r["value"] for r in rows] == [1.5, 2.5]
    assert all("time_utc" in r and "argv" in r for r in rows)
