"""SLDA self-consistency with a uniform or a learned start (all steps on the GPU).

The static SLDA state is found "iteratively via a sequence of
diagonalizations" (paper sec. "Performance of the Matrix Diagonalization
Algorithm"); each step here is one bdg_scf_step call (assembly, windowed
eigensolve, T = 0 densities, update with the pairing phase held fixed,
mixing).  The learned start replaces the uniform initial fields by the
prediction of the start-field network, trained with the library's own
kernels on converged fields produced by the same iteration.

CLI: python -m paper_2310_03341_amd.learned_start --dims 32 32 --train 64 --test 16
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import time
from typing import List, Optional

import numpy as np
import torch

from . import api, inputs
from . import checkpoint as ckpt

UNIFORM_DELTA = 0.3


def uniform_start(inst: inputs.ScfInstance, dev):
    U = torch.from_numpy(inst.Vext.copy()).to(dev)
    D = torch.full((inst.Vext.size,), UNIFORM_DELTA, dtype=torch.float64, device=dev)
    return U, D


def run_scf(stepper: api.ScfStepper, U, D, p: inputs.ScfParams, max_iter=None,
            checkpoint: Optional[str] = None, every: int = 10, fp: str = ""):
    """Iterate until the change is below p.tol; returns (iterations, converged, history).

    With `checkpoint`, the fields are written there every `every` iterations
    and at the end, and an existing checkpoint of the same problem (`fp`, see
    checkpoint.fingerprint) is continued: U and D are overwritten in place by
    its fields and the count goes on from its iteration."""
    hist = []
    max_iter = max_iter or p.max_iter
    it0 = 0
    if checkpoint:
        got = ckpt.load(checkpoint, fp)
        if got is not None:
            Uc, Dc, it0, hist = got
            U.copy_(torch.from_numpy(Uc))
            D.copy_(torch.from_numpy(Dc))
            if hist and (not math.isfinite(hist[-1]) or hist[-1] <= p.tol):
                return it0, math.isfinite(hist[-1]), hist

    def keep(it):
        if checkpoint:
            ckpt.save(checkpoint, U.cpu().numpy(), D.cpu().numpy(), it, hist, fp)

    for it in range(it0 + 1, max_iter + 1):
        change, m = stepper.step(U, D)
        hist.append(change)
        if not math.isfinite(change):
            keep(it)
            return it, False, hist
        if change <= p.tol:
            keep(it)
            return it, True, hist
        if checkpoint and it % every == 0:
            keep(it)
    keep(max(it0, max_iter))
    return max_iter, False, hist


def solve_instance(inst, p, dev, U=None, D=None, checkpoint: Optional[str] = None, every: int = 10):
    st = api.ScfStepper(inst.dims, torch.from_numpy(inst.Vext).to(dev),
                        torch.from_numpy(inst.theta).to(dev), inst.mu, p)
    if U is None:
        U, D = uniform_start(inst, dev)
    fp = ckpt.fingerprint(inst.dims, inst.mu, p, inst.Vext, inst.theta) if checkpoint else ""
    iters, ok, hist = run_scf(st, U, D, p, checkpoint=checkpoint, every=every, fp=fp)
    return iters, ok, U, D


def generate(indices: List[int], dims, p, dev, log=None, checkpoint_dir: Optional[str] = None):
    """Converged fields of the SCF instances (uniform start).  With
    `checkpoint_dir`, finished instances are kept there and not solved again,
    and the instance in progress is checkpointed every ten iterations."""
    out = []
    if checkpoint_dir:
        os.makedirs(checkpoint_dir, exist_ok=True)
    for i in indices:
        inst = inputs.scf_instance(i, dims=dims)
        t0 = time.time()
        done = os.path.join(checkpoint_dir, "instance_%d_done.npz" % i) if checkpoint_dir else None
        fp = ckpt.fingerprint(inst.dims, inst.mu, p, inst.Vext, inst.theta) if checkpoint_dir else ""
        got = ckpt.load(done, fp) if done else None
        if got is not None:
            U, D, iters, hist = got
            ok = bool(hist) and math.isfinite(hist[-1]) and hist[-1] <= p.tol
            out.append({"index": i, "inst": inst, "iters": iters, "ok": ok, "U": U, "D": D})
            if log:
                log("instance %d: from %s" % (i, done))
            continue
        partial = os.path.join(checkpoint_dir, "instance_%d_scf.npz" % i) if checkpoint_dir else None
        iters, ok, U, D = solve_instance(inst, p, dev, checkpoint=partial)
        if done:
            os.replace(partial, done)
        out.append({"index": i, "inst": inst, "iters": iters, "ok": ok,
                    "U": U.cpu().numpy(), "D": D.cpu().numpy()})
        if log:
            log("instance %d: %d iterations (%s) %.1f s" % (i, iters, "ok" if ok else "not converged",
                                                          time.time() - t0))
    return out


def _d4(a, dims, k, flip):
    """A field [ny*nx] (x fastest) under a symmetry of the square periodic
    lattice: k quarter turns, then a reflection of x.  Every lattice symmetry
    maps a trap to another valid trap and its self-consistent fields to the
    fields of that trap (the spectral kinetic term is invariant), so the
    transformed pairs are exact training data."""
    g = a.reshape(dims[1], dims[0])
    g = np.rot90(g, k)
    if flip:
        g = g[:, ::-1]
    return np.ascontiguousarray(g).ravel()


def _batch(data, idx, dev, rng=None, dims=None):
    Vs, ths, tgts = [], [], []
    for i in idx:
        V, th = data[i]["inst"].Vext, data[i]["inst"].theta
        tU, tD = data[i]["U"] - V, data[i]["D"]
        if rng is not None and dims[0] == dims[1]:
            k, f = int(rng.integers(0, 4)), bool(rng.integers(0, 2))
            V, th, tU, tD = (_d4(a, dims, k, f) for a in (V, th, tU, tD))
        Vs.append(V)
        ths.append(th)
        tgts.append(np.stack([tU, tD]))
    Vext = torch.from_numpy(np.stack(Vs)).to(dev)
    theta = torch.from_numpy(np.stack(ths)).to(dev)
    return Vext, theta, torch.from_numpy(np.stack(tgts).astype(np.float32)).to(dev)


def train(data, dims, dev, channels=32, batch=8, steps=2000, lr=2e-3, seed=0, log=None, augment=True):
    """Train the start-field network on converged fields; returns the StartNet."""
    from math import sqrt
    Nx, Ny = dims
    net = api.StartNet(channels, Ny, Nx, batch, dev)
    rng = np.random.Generator(np.random.PCG64(seed))
    # He initialisation of the flat parameter vector (weights), zero biases
    shapes = [(channels, 3), (channels, channels), (channels, channels), (2, channels)]
    vec = []
    for (o, c) in shapes:
        vec.append(rng.standard_normal(o * c * 9) * sqrt(2.0 / (9 * c)))
        vec.append(np.zeros(o))
    vec[-2] *= 0.1
    net.params.copy_(torch.from_numpy(np.concatenate(vec).astype(np.float32)))
    mu = data[0]["inst"].mu
    n = len(data)
    for step in range(steps):
        idx = rng.choice(n, size=batch, replace=n < batch)
        Vext, theta, tgt = _batch(data, idx, dev, rng if augment else None, dims)
        loss = net.backward(Vext, theta, mu, tgt)
        net.adam(lr * (0.1 if step > 0.75 * steps else 1.0))
        if log and (step % 500 == 0 or step == steps - 1):
            log("step %d loss %.3e" % (step, loss.item()))
    return net


def predict_start(net: api.StartNet, inst, dev):
    B = net.shape.batch
    Vext = torch.from_numpy(np.stack([inst.Vext] * B)).to(dev)
    theta = torch.from_numpy(np.stack([inst.theta] * B)).to(dev)
    y = net.forward(Vext, theta, inst.mu)
    return net.start_fields(y, 0, torch.from_numpy(inst.Vext).to(dev))


def evaluate(net, test, p, dev, log=None):
    """SCF iterations from uniform vs learned start and the converged-field difference."""
    rows = []
    for d in test:
        inst = d["inst"]
        U, D = predict_start(net, inst, dev)
        it_l, ok_l, Ul, Dl = solve_instance(inst, p, dev, U, D)
        if not ok_l:  # fallback: the uniform start
            it_l2, ok_l, Ul, Dl = solve_instance(inst, p, dev)
            it_l += it_l2
        du = float(np.sqrt(np.mean((Ul.cpu().numpy() - d["U"]) ** 2)))
        dd = float(np.sqrt(np.mean((Dl.cpu().numpy() - d["D"]) ** 2)))
        rows.append({"index": d["index"], "iters_uniform": d["iters"], "iters_learned": it_l,
                     "converged": ok_l, "l2_dU": du, "l2_dDelta": dd})
        if log:
            log("test %d: uniform %d, learned %d iterations" % (d["index"], d["iters"], it_l))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=int, nargs=2, default=[32, 32])
    ap.add_argument("--train", type=int, default=64)
    ap.add_argument("--test", type=int, default=16)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--channels", type=int, default=32)
    ap.add_argument("--alpha", type=float, default=0.9, help="linear mixing (same for both starts)")
    ap.add_argument("--max-iter", type=int, default=400)
    ap.add_argument("--out", type=str, default="")
    ap.add_argument("--checkpoint-dir", type=str, default="",
                    help="keep converged instances (and the one in progress) here; a rerun continues")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    p = dataclasses.replace(inputs.ScfParams(), alpha=args.alpha, max_iter=args.max_iter)
    dims = tuple(args.dims)
    log = lambda s: print(s, flush=True)  # noqa: E731
    t0 = time.time()
    # instances whose uniform-start iteration does not converge (limit cycles
    # of a level on the window edge) are left out of both sets
    cdir = args.checkpoint_dir or None
    train_all = generate(list(range(args.train)), dims, p, dev, log, checkpoint_dir=cdir)
    test_all = generate(list(range(10000, 10000 + args.test)), dims, p, dev, log, checkpoint_dir=cdir)
    train_set = [d for d in train_all if d["ok"]]
    test_set = [d for d in test_all if d["ok"]]
    t1 = time.time()
    net = train(train_set, dims, dev, channels=args.channels, steps=args.steps, log=log)
    t2 = time.time()
    rows = evaluate(net, test_set, p, dev, log)
    iu = np.mean([r["iters_uniform"] for r in rows])
    il = np.mean([r["iters_learned"] for r in rows])
    res = {"dims": list(dims), "train": len(train_set), "test": len(test_set), "alpha": p.alpha,
           "dropped_not_converged": (len(train_all) - len(train_set), len(test_all) - len(test_set)),
           "mean_iters_uniform": iu, "mean_iters_learned": il,
           "max_l2_dU": max(r["l2_dU"] for r in rows), "max_l2_dDelta": max(r["l2_dDelta"] for r in rows),
           "gen_s": t1 - t0, "train_s": t2 - t1, "rows": rows}
    print(json.dumps({k: v for k, v in res.items() if k != "rows"}))
    if args.out:
        json.dump(res, open(args.out, "w"), indent=1)


if __name__ == "__main__":
    main()
