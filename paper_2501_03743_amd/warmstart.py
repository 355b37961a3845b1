"""Learned warm start for the s-step solver.

A 3-level U-shaped conv net (the library's ssp_net_*: BF16 matrix-core
convolutions with FP32 accumulation, FP32 master weights, Adam) maps the
coefficient field and source of a variable-coefficient Poisson problem
-div(k grad u) = f to an initial guess x0.  Its training targets are
solutions computed by the library's own solver.  At inference the guess goes
to ssp_solve with warm_start = 1 and a few damped Jacobi sweeps: the sweeps
remove the rough part of the guess's error (BF16 noise, which the operator
amplifies), then the solver judges it by its true residual and starts from
x0 = 0 instead when ||b - A x0|| >= ||b||.  Training minimises the error's
energy e^T (L + lam I) e (L the 7-point Laplacian) rather than its mean
square: that is the norm CG pays for when it starts from the guess.

Normalisation: the input channels are log k and f / rms(f); the target is
u / (rms(f) * c) with one constant c (the RMS of u / rms(f) over the training
set).  Since u is linear in f for a fixed k, the prediction is rescaled by
rms(f) * c.

This module only marshals tensors: every network and solver step runs in the
library's kernels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from . import sstep
from . import workloads as wl


def features(logk, f, shape):
    """Network input [D, H, W, 2] float32 and the source scale rms(f)."""
    import torch
    nx, ny, nz = shape
    fs = float(torch.sqrt(torch.mean(f * f)))
    fs = fs if fs > 0.0 else 1.0
    inp = torch.stack([logk, f / fs], dim=-1).to(torch.float32).reshape(nz, ny, nx, 2)
    return inp, fs


@dataclass
class WarmStartData:
    inputs: "object"          # float32 [N, D, H, W, 2] (device)
    targets: "object"         # float32 [N, D, H, W], u / rms(f)
    seeds: List[int]
    outer: List[int] = field(default_factory=list)
    solve_ms: List[float] = field(default_factory=list)


def generate(H: "sstep.Handle", shape, seeds, s: int = 4, rtol: float = 1e-8,
             log: Optional[Callable[[str], None]] = None) -> WarmStartData:
    """Solves one problem per seed with the s-step solver (x0 = 0) and keeps
    (features, solution) pairs on the device."""
    import torch
    nx, ny, nz = shape
    N = len(seeds)
    inputs = torch.empty((N, nz, ny, nx, 2), device="cuda", dtype=torch.float32)
    targets = torch.empty((N, nz, ny, nx), device="cuda", dtype=torch.float32)
    data = WarmStartData(inputs, targets, list(seeds))
    t_last = time.time()
    for i, seed in enumerate(seeds):
        logk, k, f, b = wl.warm_start_problem(shape, seed)
        A = H.matrix_stencil("3d7_vark", shape, k=k)
        x = torch.zeros_like(b)
        t0 = time.perf_counter()
        r = H.solve(A, b, x, s=s, rtol=rtol)
        data.solve_ms.append(1e3 * (time.perf_counter() - t0))
        A.close()
        if r.status != sstep.OK:
            raise RuntimeError("training solve %d did not converge (status %d)" % (seed, r.status))
        data.outer.append(r.outer)
        inp, fs = features(logk, f, shape)
        inputs[i] = inp
        targets[i] = (x / fs).to(torch.float32).reshape(nz, ny, nx)
        if log and (time.time() - t_last > 20 or i + 1 == N):
            t_last = time.time()
            log("generated %d/%d (last: %d outer iterations, %.1f ms)"
                % (i + 1, N, r.outer, data.solve_ms[-1]))
    return data


class WarmStart:
    """The warm-start model: the library's network plus the output scale."""

    def __init__(self, H: "sstep.Handle", shape, batch: int = 4, seed: int = 0):
        self.H = H
        self.shape = tuple(shape)
        nx, ny, nz = self.shape
        self.batch = batch
        self.net = H.net((nz, ny, nx), max_batch=batch, seed=seed)
        self.out_scale = 1.0
        self.history: List[float] = []

    def fit(self, data: WarmStartData, epochs: int, lr: float = 2e-3, seed: int = 0,
            log: Optional[Callable[[str], None]] = None, time_limit: float = 0.0,
            loss: str = "h1", lam: float = 1e-3):
        """Adam on normalised targets with a cosine-decayed learning rate and
        shuffled mini-batches (seeded).  loss "h1": the error's energy
        e^T (L + lam I) e (L the 7-point Laplacian), which is what CG pays
        for when it starts from the prediction; "mse": the mean square."""
        import torch
        N = data.inputs.shape[0]
        self.out_scale = float(torch.sqrt(torch.mean(data.targets.double() ** 2)))
        if not self.out_scale > 0.0:
            self.out_scale = 1.0
        B = self.batch
        steps_per_epoch = N // B
        if steps_per_epoch < 1:
            raise ValueError("need at least one full batch of training samples")
        total = epochs * steps_per_epoch
        g = np.random.default_rng(seed)
        xb = torch.empty((B,) + tuple(data.inputs.shape[1:]), device="cuda", dtype=torch.float32)
        tb = torch.empty((B,) + tuple(data.targets.shape[1:]), device="cuda", dtype=torch.float32)
        y = torch.empty_like(tb)
        inv = 1.0 / self.out_scale
        step = 0
        t0 = time.time()
        t_last = t0
        for ep in range(epochs):
            perm = torch.from_numpy(g.permutation(N)).cuda()
            acc = 0.0
            for j in range(steps_per_epoch):
                idx = perm[j * B:(j + 1) * B]
                torch.index_select(data.inputs, 0, idx, out=xb)
                torch.index_select(data.targets, 0, idx, out=tb)
                tb.mul_(inv)
                self.net.forward(xb, y)
                if loss == "h1":
                    lval, dy = self.net.loss_h1(y, tb, lam)
                else:
                    lval, dy = self.net.loss(y, tb)
                self.net.zero_grad()
                self.net.backward(dy)
                lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * step / total))
                self.net.adam_step(lr_t)
                acc += lval
                step += 1
            self.history.append(acc / steps_per_epoch)
            if log and (time.time() - t_last > 20 or ep + 1 == epochs):
                t_last = time.time()
                log("epoch %d/%d: loss %.4e (%.1f s)" % (ep + 1, epochs, self.history[-1],
                                                         time.time() - t0))
            if time_limit and time.time() - t0 > time_limit:
                break
        return self.history

    def predict(self, logk, f, out=None):
        """x0 (float64, n) for one problem: features, network and output
        scaling in one library call (the same values as `features`, a batch-1
        forward and y * rms(f) * out_scale)."""
        return self.net.predict(logk.reshape(-1), f.reshape(-1), self.out_scale, out=out)

    def close(self):
        self.net.close()


@dataclass
class EvalRecord:
    seed: int
    outer_zero: int
    outer_warm: int
    outer_smoothed_zero: int  # control: x0 = 0 with the same smoothing sweeps
    ms_zero: float
    ms_warm: float            # network forward + sweeps + judge + solve
    rel0: float               # ||b - A x0|| / ||b|| of the (smoothed) prediction
    kept: int                 # 1: warm start used, 0: fell back to x0 = 0
    true_zero: float
    true_warm: float


def evaluate(H: "sstep.Handle", model: WarmStart, seeds, s: int = 4, rtol: float = 1e-8,
             precision: str = "fp64", sweeps: int = 16) -> List[EvalRecord]:
    """Held-out comparison: the same solve from x0 = 0, from the network's
    guess (smoothed by `sweeps` damped Jacobi sweeps and judged by the
    solver), and, as a control, from x0 = 0 smoothed by the same sweeps.
    Times are end to end on the device (the warm time includes inference)."""
    import torch
    out = []
    for seed in seeds:
        logk, k, f, b = wl.warm_start_problem(model.shape, seed)
        A = H.matrix_stencil("3d7_vark", model.shape, k=k)
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r0 = H.solve(A, b, x, s=s, rtol=rtol, precision=precision)
        t1 = time.perf_counter()
        x.zero_()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        model.predict(logk, f, out=x)
        r1 = H.solve(A, b, x, s=s, rtol=rtol, precision=precision, warm_start=True,
                     warm_sweeps=sweeps)
        t3 = time.perf_counter()
        x.zero_()
        rc = H.solve(A, b, x, s=s, rtol=rtol, precision=precision, warm_start=True,
                     warm_sweeps=sweeps)
        A.close()
        out.append(EvalRecord(seed, r0.outer, r1.outer, rc.outer, 1e3 * (t1 - t0),
                              1e3 * (t3 - t2), r1.warm_rel0, r1.warm_kept, r0.true_rel,
                              r1.true_rel))
    return out


def summarize(records: List[EvalRecord]) -> dict:
    oz = np.array([r.outer_zero for r in records], dtype=float)
    ow = np.array([r.outer_warm for r in records], dtype=float)
    oc = np.array([r.outer_smoothed_zero for r in records], dtype=float)
    tz = np.array([r.ms_zero for r in records])
    tw = np.array([r.ms_warm for r in records])
    return {
        "n": len(records),
        "outer_zero_mean": float(oz.mean()), "outer_warm_mean": float(ow.mean()),
        "outer_smoothed_zero_mean": float(oc.mean()),
        "iteration_gain": float(1.0 - ow.sum() / oz.sum()),
        "iteration_gain_vs_smoothed_zero": float(1.0 - ow.sum() / oc.sum()),
        "ms_zero_mean": float(tz.mean()), "ms_warm_mean": float(tw.mean()),
        "time_gain": float(1.0 - tw.sum() / tz.sum()),
        "fallbacks": int(sum(1 for r in records if r.kept == 0)),
        "rel0_median": float(np.median([r.rel0 for r in records])),
        "true_rel_max_zero": float(max(r.true_zero for r in records)),
        "true_rel_max_warm": float(max(r.true_warm for r in records)),
        "worse_count": int(np.sum(ow > oz)),
    }
