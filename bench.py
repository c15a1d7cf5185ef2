"""Benchmark: dense BdG diagonalisation on one MI355X.

A step is one pass of the hot path on one synthetic BdG matrix: assembly of
H (eq. stHpsi) on the GPU, then the full FP64 two-stage eigensolver
(dense -> band -> tridiagonal -> divide and conquer -> both back-transforms)
returning every eigenpair.  The default workload is the 24x24x24 lattice with
a vortex line (n = 27648).  The reported value is the eigensolver time in
seconds per matrix (lower is better); TFLOP/s uses the two-stage algorithmic
count F = (16/3 + 4/3) n^3 + 16 n^2 m.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--dims 24 24 24]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6e12
PEAK_HBM = 8.0e12

# HBM traffic of one bt2_apply launch from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes (KiB per dispatch), each scaled by what the same counter reads for a
# 1 GiB device copy in the same run.  Valid only for the kernel source it was
# measured on (sha256 of csrc/bt2.hip) and the same workload; otherwise the
# bench reports null.
BT2_TRAFFIC = {"sha256": "261b228058abb244f85f7984d0fdc73869bf35f5faa24088de71b1f9b2bedba0",
               "n": 27648, "m_bt": 13824, "fetch_bytes": 2726300789783.9, "write_bytes": 2644665558752.0}


def _bt2_source_sha() -> str:
    import hashlib
    with open(os.path.join(ROOT, "paper_2310_03341_amd", "csrc", "bt2.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def bt2_traffic(n: int, m_bt: int):
    t = BT2_TRAFFIC
    if not t or t["sha256"] != _bt2_source_sha() or t["n"] != n or t["m_bt"] != m_bt:
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def flops_two_stage(n: int, m: int) -> float:
    return (16.0 / 3.0 + 4.0 / 3.0) * n ** 3 + 16.0 * n * n * m


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(budget_s: float = 20.0):
    """Time the CPU oracle (Householder + QL, all eigenpairs) on a bounded
    sample of the same generator and scale it to the metric's matrix by n^3."""
    import numpy as np

    import oracle
    from paper_2310_03341_amd import inputs
    oracle.build()
    cores = len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    dims = (8, 8, 8)
    w = inputs.line_3d(dims, instance=0, config=2)
    H = oracle.assemble_workload(w)
    t0 = time.perf_counter()
    oracle.eigh_hqr(H, vectors=True)
    dt = time.perf_counter() - t0
    # grow the sample while it stays inside the time budget
    for dims in ((10, 10, 8), (12, 12, 8), (12, 12, 12)):
        n_next = 2 * int(np.prod(dims))
        if dt * (n_next / H.shape[0]) ** 3 > budget_s:
            break
        w = inputs.line_3d(dims, instance=0, config=2)
        H = oracle.assemble_workload(w)
        t0 = time.perf_counter()
        oracle.eigh_hqr(H, vectors=True)
        dt = time.perf_counter() - t0
    n_s = H.shape[0]
    # a second, half-size sample gives the measured exponent of the growth
    w2 = inputs.line_3d(tuple(max(2, d // 2) if i == 0 else d for i, d in enumerate(w.dims)), instance=0, config=2)
    H2 = oracle.assemble_workload(w2)
    t0 = time.perf_counter()
    oracle.eigh_hqr(H2, vectors=True)
    dt2 = time.perf_counter() - t0
    expo = math.log(dt / dt2) / math.log(n_s / H2.shape[0]) if dt2 > 0 else float("nan")
    fit = "measured growth exponent %.2f between n=%d (%.2f s) and n=%d" % (expo, H2.shape[0], dt2, n_s)
    return dt, n_s, cores, "x".join(str(v) for v in w.dims), fit


def sample_pairs(W, Z, nsample=256, seed=0):
    """Host copies of sampled eigenpairs (ends of the spectrum, around E = 0,
    random columns) for the host certification."""
    import numpy as np
    import torch
    n = Z.shape[1]
    rng = np.random.default_rng(seed)
    h = n // 2
    idx = np.unique(np.r_[0, 1, n - 2, n - 1, max(h - 2, 0):min(h + 2, n), rng.choice(n, min(n, nsample), False)])
    idx = idx[:nsample]
    return W.cpu().numpy(), idx, Z[:, torch.from_numpy(idx).to(Z.device)].cpu().numpy()


def certify_sampled(w, sample):
    """max_j ||H z_j - w_j z_j|| / max|w| and max |(Z_s^H Z_s - I)| over the
    sampled columns, in FP64 on the host with the oracle's matrix-free H."""
    import numpy as np

    import oracle
    Wh, idx, Zs = sample
    R = oracle.apply_h(w.dims, w.U, w.Delta, w.mu, Zs) - Zs * Wh[idx]
    res = float(np.linalg.norm(R, axis=0).max() / np.abs(Wh).max())
    gram = float(np.abs(Zs.conj().T @ Zs - np.eye(idx.size)).max())
    return {"columns": int(idx.size), "max_resid": res, "gram_defect": gram}


def check_blocked(api, torch, H, W, Z, block=8192):
    """Residual and Gram defect of (W, Z) column block by column block, so that
    no n x m scratch is needed: residual per block through bdg_check, the Gram
    matrix block pair by block pair through the library's ZGEMM."""
    n, m = Z.shape
    res = 0.0
    gram = 0.0
    # bdg_check scales by the largest |w| it is given: rescale each block to
    # ||H||_2 (max |w| when the whole spectrum was solved; for a window, the
    # larger of that and a power-iteration estimate)
    normH = float(W.abs().max())
    if m < n:
        torch.manual_seed(3)
        X = api.colmajor(n, 4, torch.complex128, Z.device)
        X.copy_(torch.randn(n, 4, dtype=torch.complex128, device=Z.device))
        Y = api.colmajor(n, 4, torch.complex128, Z.device)
        est = 0.0
        for _ in range(40):
            X /= X.norm(dim=0, keepdim=True)
            api.zgemm("N", "N", H, X, Y)
            est = float(Y.norm(dim=0).max())
            X, Y = Y, X
        normH = max(normH, est)
        del X, Y
    for j0 in range(0, m, block):
        j1 = min(m, j0 + block)
        print("[bench] check columns %d..%d" % (j0, j1), file=sys.stderr, flush=True)
        r, g = api.check(H, W[j0:j1], Z[:, j0:j1])
        res = max(res, r * float(W[j0:j1].abs().max()) / normH)
        gram = max(gram, g)
        for i0 in range(0, j0, block):
            i1 = min(m, i0 + block)
            G = api.colmajor(i1 - i0, j1 - j0, torch.complex128, Z.device)
            api.zgemm("C", "N", Z[:, i0:i1], Z[:, j0:j1], G)
            gram = max(gram, float(G.abs().max()))
            del G
    return res, gram


def bench_tdslda(api, inputs, torch, dev, progress, dims=(16, 16, 16), steps=20):
    """TDSLDA evolution (eq. TDSLDA, fifth-order ABM) of the quasiparticle
    states 0 < E < pi^2/2 of a vortex-line BdG matrix on a 16^3 lattice (the
    largest whose states fit the LDS-staged kernel), self-consistent fields
    after a 10 % quench of the potential.  Timed over `steps` ABM steps after
    the four RK4 start steps, with HIP events on the library's stream.  A step
    moves 18 state arrays (16 n m bytes each) through HBM."""
    w = inputs.line_3d(dims, instance=0, config=2)
    n = w.n
    progress("TDSLDA: diagonalising the %s start (n=%d)" % ("x".join(map(str, dims)), n))
    U = torch.from_numpy(w.U).to(dev)
    D = torch.from_numpy(w.Delta).to(dev)
    H = api.colmajor(n, n, torch.complex128, dev)
    api.assemble(w.dims, U, D, w.mu, out=H)
    solver = api.Solver(n, api.make_opts(ph_mirror=1), dev)
    W, Z = solver(H, 4.9406564584124654e-324, math.pi ** 2 / 2)
    m = W.numel()
    Phi = api.colmajor(n, m, torch.complex128, dev)
    Phi.copy_(Z)
    del solver, H, Z
    torch.cuda.empty_cache()
    p = inputs.ScfParams()
    Vq = U * 1.1
    ev = api.TdEvolver(w.dims, m, w.mu, p.B, p.g, Vext=Vq, self_consistent=True, device=dev)
    dt = 0.004
    ev.evolve(Phi, dt, 4)  # RK4 start; fills the history
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ev.evolve(Phi, dt, steps)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / steps
    nbytes = 18.0 * 16.0 * n * m
    gram = api.colmajor(m, m, torch.complex128, dev)
    api.zgemm("C", "N", Phi, Phi, gram)
    eye = torch.eye(m, dtype=torch.complex128, device=dev)
    defect = float((gram - eye).abs().max())
    progress("TDSLDA: %d states, %.3f ms per step" % (m, 1e3 * t))
    return {"workload": "TDSLDA %s vortex line, n=%d, %d states 0<E<pi^2/2, ABM5 dt=%g" % (
                "x".join(map(str, dims)), n, m, dt),
            "ms_per_step": round(1e3 * t, 4), "steps": steps,
            "roofline": {"bound": "hbm", "achieved": round(nbytes / t / 1e9, 1), "peak": 8000.0, "unit": "GB/s",
                         "frac": round(nbytes / t / PEAK_HBM, 4), "bytes_per_step": nbytes},
            "gram_defect_after": defect}


def bench_onestage(api, inputs, torch, dev, progress, dims=(24, 24, 24)):
    """The one-stage solver (bdg_eigh1) on the metric workload: the complex
    vortex-line matrix, and a real symmetric BdG matrix of the same order and
    fields with a real gap |Delta| (the paper's own benchmark is ELPA's
    one-stage solver on real matrices; it states complex takes about twice as
    long).  All eigenpairs, one solve each, times from the library's events."""
    import numpy as np
    w = inputs.metric_3d() if dims == (24, 24, 24) else inputs.line_3d(dims, instance=0, config=2)
    n = w.n
    out = {"workload": "one-stage FP64, %s vortex line, n=%d, all eigenpairs" % ("x".join(map(str, dims)), n)}
    U = torch.from_numpy(w.U).to(dev)
    for kind in ("complex", "real"):
        D = torch.from_numpy(w.Delta if kind == "complex" else np.abs(w.Delta).astype(np.complex128)).to(dev)
        Hc = api.colmajor(n, n, torch.complex128, dev)
        api.assemble(w.dims, U, D, w.mu, out=Hc)
        if kind == "real":
            A = api.colmajor(n, n, torch.float64, dev)
            A.copy_(Hc.real)
            del Hc
        else:
            A = Hc
        torch.cuda.empty_cache()
        progress("one-stage %s solve, n=%d" % (kind, n))
        W, Z, rep = api.eigh1(A)
        torch.cuda.synchronize()
        out[kind + "_s"] = round(rep.stage_ms[7] / 1e3, 3)
        out[kind + "_stage_ms"] = {"tridiag": round(rep.stage_ms[0], 1), "stedc": round(rep.stage_ms[2], 1),
                                   "back": round(rep.stage_ms[4], 1)}
        del A, W, Z
        torch.cuda.empty_cache()
    out["complex_over_real"] = round(out["complex_s"] / out["real_s"], 3)
    return out


def bench_int8_gemm(api, torch, dev, progress, M=8192, N=8192, K=8192, slices=8, reps=3):
    """Complex C = A^H B emulated on the INT8 matrix cores (bdg_gemm_int8) next to
    the FP64 MFMA ZGEMM (bdg_zgemm) on the same operands; rates count 8MNK."""
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3
    torch.manual_seed(0)
    A = api.colmajor(K, M, torch.complex128, dev)
    A.copy_(torch.randn(K, M, dtype=torch.complex128, device=dev))
    B = api.colmajor(K, N, torch.complex128, dev)
    B.copy_(torch.randn(K, N, dtype=torch.complex128, device=dev))
    C64 = api.colmajor(M, N, torch.complex128, dev)
    C8 = api.colmajor(M, N, torch.complex128, dev)
    progress("int8-emulated ZGEMM %dx%dx%d, %d slices" % (M, N, K, slices))
    t64 = timed(lambda: api.zgemm("C", "N", A, B, C64))
    t8 = timed(lambda: api.gemm_int8("C", "N", A, B, C8, slices=slices))
    fl = 8.0 * M * N * K
    return {"shape": [M, N, K], "slices": slices, "int8_s": round(t8, 4), "fp64_s": round(t64, 4),
            "int8_tflops_equiv": round(fl / t8 / 1e12, 1), "fp64_tflops": round(fl / t64 / 1e12, 1),
            "max_rel_diff": float((C8 - C64).abs().max() / C64.abs().max())}


def bench_bt2_alone(api, torch, dev, progress, n=27648, m=13824, band=64):
    """The back-transformation 2 alone at the solver's shape (n = 27648, the
    13824 back-transformed columns of the particle-hole mirror), for counter
    runs that must not go through stage 2's launch loop.  Reflectors are
    synthetic with tau = 0: the apply kernel's loads, products and stores do
    not depend on the values, and Z stays finite.  One call of the stage."""
    import numpy as np
    torch.manual_seed(0)
    T = (n - 2 - np.arange(n - 2, dtype=np.int64)) // band + 1
    voff_h = np.zeros(n + 1, dtype=np.int64)
    voff_h[1:n - 2] = np.cumsum(T)[:-1]
    nrefl = int(T.sum())
    voff = torch.from_numpy(voff_h).to(dev)
    V2 = (torch.randn((nrefl + 1) * band, dtype=torch.complex128, device=dev) * 0.02)
    tau2 = torch.zeros(nrefl + 1, dtype=torch.float64, device=dev)
    e = torch.randn(n, dtype=torch.complex128, device=dev)
    Y = api.colmajor(n, n, torch.float64, dev)
    Y.copy_(torch.randn(n, n, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    progress("back-transformation 2 alone, n=%d, %d columns" % (n, m))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    Z = api.stage_bt2(e, Y, n - m, m, V2, tau2, voff, band, rowmajor=True)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3
    return {"n": n, "m_bt": m, "band": band, "stage_s": round(t, 4), "finite": bool(torch.isfinite(Z).all())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", type=int, nargs="+", default=[24, 24, 24])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--check", action="store_true", help="FP64 residual/Gram check of the last step")
    ap.add_argument("--no-ph-mirror", action="store_true",
                    help="back-transform every eigenvector instead of the E > 0 half + mirror")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32+refinement arm")
    ap.add_argument("--window", type=float, nargs=2, default=None, metavar=("EMIN", "EMAX"),
                    help="eigenvalue window (default: all eigenpairs)")
    ap.add_argument("--max-pairs", type=int, default=0,
                    help="mixed arm: most eigenpairs the window may hold (sizes the refinement buffers; 0 = n)")
    ap.add_argument("--zcols", type=float, default=1.0,
                    help="columns of Z to allocate, as a fraction of n (a window needs fewer)")
    ap.add_argument("--no-td", action="store_true", help="skip the TDSLDA and INT8-GEMM side measurements")
    ap.add_argument("--no-onestage", action="store_true", help="skip the one-stage (real and complex) solves")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device copy (read 1 GiB, write 1 GiB) before the solves, "
                         "as the reference point for HBM byte counters")
    ap.add_argument("--only", choices=["tdslda", "onestage", "int8gemm", "bt2"], default=None,
                    help="run one side measurement alone and print its JSON (for profiling)")
    ap.add_argument("--jsonl", type=str, default="",
                    help="also append the result line, with a UTC time stamp and the command line, "
                         "to this JSON-lines log")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver is single-GPU; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    # the library's stage lines keep a long solve visibly alive
    os.environ.setdefault("BDG_VERBOSE", "1")
    import torch

    from paper_2310_03341_amd import api, inputs

    dev = torch.device("cuda:0")
    dims = tuple(args.dims)
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)  # one elementwise kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        del src, dst
    if args.only:
        def say(msg):
            print("[bench] " + msg, file=sys.stderr, flush=True)
        if args.only == "tdslda":
            res = bench_tdslda(api, inputs, torch, dev, say)
        elif args.only == "onestage":
            res = bench_onestage(api, inputs, torch, dev, say, dims)
        elif args.only == "bt2":
            res = bench_bt2_alone(api, torch, dev, say)
        else:
            res = bench_int8_gemm(api, torch, dev, say)
        print(json.dumps({args.only: res}))
        append_log(args.jsonl, {args.only: res})
        return
    if dims == (24, 24, 24):
        w = inputs.metric_3d()
    elif dims == (32, 32, 24):
        w = inputs.precision_3d()
    elif dims == (32, 32, 32):
        w = inputs.ring_3d()
    else:
        w = inputs.line_3d(dims, instance=0, config=2)
    n = w.n
    U = torch.from_numpy(w.U).to(dev)
    D = torch.from_numpy(w.Delta).to(dev)
    H = api.colmajor(n, n, torch.complex128, dev)
    ph = 0 if args.no_ph_mirror else 1
    opts = api.make_opts(ph_mirror=ph)
    solver = api.Solver(n, opts, dev)
    W = torch.empty(n, dtype=torch.float64, device=dev)
    zc = max(1, min(n, int(math.ceil(args.zcols * n))))
    Z = api.colmajor(n, zc, torch.complex128, dev)
    lo, hi = (-math.inf, math.inf) if args.window is None else tuple(args.window)

    def step():
        api.assemble(w.dims, U, D, w.mu, out=H)
        return solver(H, lo, hi, W, Z)

    def progress(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    progress("n=%d, workload %s" % (n, w.name))
    for _ in range(args.warmup):
        step()
        torch.cuda.synchronize()
        progress("warmup step %.2f s" % (solver.report.stage_ms[7] / 1e3))
    torch.cuda.synchronize()
    stage = [0.0] * 8
    t_eigh = []
    t_bt2 = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Wk, Zk = step()
        rep = solver.report
        t_eigh.append(rep.stage_ms[7] / 1e3)
        t_bt2.append(rep.bt2_kernel_ms / 1e3)
        for i in range(8):
            stage[i] += rep.stage_ms[i] / args.steps
        progress("timed step %.2f s" % (rep.stage_ms[7] / 1e3))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sample64 = sample_pairs(Wk, Zk) if not args.no_cpu else None
    sample_mixed = None
    m = Wk.numel()
    ms_step = 1e3 * wall / args.steps
    t_solve = sum(t_eigh) / len(t_eigh)
    # back-transformed columns: with the mirror, only the E > 0 half of a window
    # that holds the partners of all its E < 0 eigenvalues
    neg = int((Wk < 0).sum())
    mirrored = bool(ph) and 0 < neg <= m - neg
    m_bt = m - neg if mirrored else m
    F = flops_two_stage(n, m_bt)
    # dominant kernel: the back-transformation-2 apply kernel (one launch per solve)
    t_k = sum(t_bt2) / len(t_bt2)
    f_k = 8.0 * n * n * m_bt
    out = {
        "metric": "BdG eigh time (s) + FP64-matrix TFLOP/s at n=27648; mixed+refined vs FP64",
        "value": round(t_solve, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "BdG %s (%s), n=%d, %s: %d eigenpairs, FP64 two-stage" % (
                       "x".join(map(str, dims)), w.name,  n,
                       "all" if args.window is None else "window [%g, %g]" % (lo, hi), m),
                   "n": n, "m": m, "ph_mirror": bool(ph), "mirrored": mirrored,
                   "flop_model": "(16/3+4/3) n^3 + 16 n^2 m_bt, m_bt = %d back-transformed columns" % m_bt},
        "tflops": round(F / t_solve / 1e12, 3),
        "frac_fp64_peak": round(F / t_solve / PEAK_FP64_MFMA, 4),
        "stage_ms": {k: round(v, 2) for k, v in zip(
            ["he2hb", "hb2st", "stedc", "bt2", "bt1", "refine", "select", "total"], stage)},
        "roofline": {"kernel": "bt2_apply", "bound": "mfma", "achieved": round(f_k / t_k / 1e12, 3),
                     "peak": 78.6, "unit": "TFLOP/s", "frac": round(f_k / t_k / PEAK_FP64_MFMA, 4),
                     "traffic": bt2_traffic(n, m_bt), "flops_per_launch": f_k,
                     "ms_per_launch": round(1e3 * t_k, 2)},
    }
    if args.check:
        # the FP64 solve destroyed H: assemble it again into the same buffer
        api.assemble(w.dims, U, D, w.mu, out=H)
        res, gram = check_blocked(api, torch, H, Wk, Zk)
        out["max_resid"] = res
        out["gram_defect"] = gram
    if not args.no_mixed:
        # the precision arm on the same matrix: FP32 reduction + FP64 refinement
        W64 = Wk.clone()
        del solver
        torch.cuda.empty_cache()
        mopts = api.make_opts(precision=api.BDG_FP32_REFINED, ph_mirror=ph, max_pairs=args.max_pairs)
        msolver = api.Solver(n, mopts, dev)
        api.assemble(w.dims, U, D, w.mu, out=H)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Wm, Zm = msolver(H, lo, hi, W, Z)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t0
        rep = msolver.report
        if not args.no_cpu:
            sample_mixed = sample_pairs(Wm, Zm)
        mixed = {"time_s": round(rep.stage_ms[7] / 1e3, 4), "wall_s": round(tm, 3),
                 "refine_iters": rep.refine_iters, "refine_defect": rep.max_resid,
                 "close_pairs_step1": rep.refine_close_pairs, "clustered_cols_step1": rep.refine_cluster_cols,
                 "stage_ms": {k: round(v, 2) for k, v in zip(
                     ["he2hb32", "hb2st32", "stedc", "bt2_32", "bt1_32", "refine64", "select", "total"],
                     list(rep.stage_ms))}}
        if args.check:
            # the mixed solve reads H but keeps it (the FP64 refinement needs it)
            res, gram = check_blocked(api, torch, H, Wm, Zm)
            mixed["max_resid"] = res
            mixed["gram_defect"] = gram
        if Wm.numel() == W64.numel():
            mixed["max_eig_diff_vs_fp64"] = float((Wm - W64).abs().max())
        out["mixed_refined"] = mixed
        progress("mixed arm %.2f s" % mixed["time_s"])
        del msolver
    if not args.no_td:
        out["tdslda"] = bench_tdslda(api, inputs, torch, dev, progress)
    if not args.no_td:
        out["int8_gemm"] = bench_int8_gemm(api, torch, dev, progress)
    if not args.no_onestage:
        del H
        torch.cuda.empty_cache()
        out["one_stage"] = bench_onestage(api, inputs, torch, dev, progress, dims)
        out["one_stage"]["two_stage_complex_s"] = out["value"]
    if not args.no_cpu:
        progress("CPU oracle baseline")
        dt, n_s, cores, sdims, fit = cpu_baseline()
        scale = (n / n_s) ** 3
        out["cpu_baseline"] = {"value": round(dt * scale, 1), "unit": "s", "cores": cores,
                               "kind": "oracle",
                               "sample": "oracle Householder+QL, all eigenpairs, %s lattice "
                                         "(n=%d) in %.1f s, scaled by (n/%d)^3; %s" % (sdims, n_s, dt, n_s, fit),
                               "cpu": cpu_model()}
        # FP64 certification of sampled eigenpairs of the timed solve on the
        # host: residuals with the oracle's matrix-free H, Gram matrix in numpy
        progress("host FP64 certification of sampled eigenpairs")
        out["cpu_certification"] = {"fp64": certify_sampled(w, sample64)}
        if sample_mixed is not None:
            out["cpu_certification"]["mixed_refined"] = certify_sampled(w, sample_mixed)
    print(json.dumps(out))
    append_log(args.jsonl, out)


def append_log(path, rec):
    """One JSON line per run appended to `path` (no-op for an empty path)."""
    if not path:
        return
    import datetime
    row = {"time_utc": datetime.datetime.now(datetime.timezone.utc).isoformat(timespec="seconds"),
           "argv": sys.argv[1:]}
    row.update(rec)
    with open(path, "a") as f:
        f.write(json.dumps(row) + "\n")


if __name__ == "__main__":
    main()
