#!/usr/bin/env python3
"""Time-to-solution of preconditioned s-step CG on one MI355X.

Workload (one "step" = one full solve): 3D 7-point constant-coefficient
Poisson on a 128^3 grid (n = 2,097,152, Dirichlet), FP64 CSR, Jacobi
preconditioner, s = 4, b ~ N(0, 1) from seed 0, x0 = 0, rtol 1e-8.  Inputs
are resident in HBM before the timed region.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Besides the timed solves the line carries: the matrix-powers kernel's
achieved bandwidth against the 8 TB/s HBM peak (algorithmic bytes per launch
over the mean launch time from HIP events on the library's stream) at 128^3,
where the matrix stays in the memory-side cache, and at 256^3, where it is
streamed from HBM; the bandwidth of the library's own streaming read and copy
kernels; the comparison rows of every workload (standard PCG, PFCG, each s,
the matrix-free form, the Chebyshev basis, mixed precision); the 27-point
256^3 problem against the oracle's FP64 solution; the batch of 32 uneven
systems; a bounded run of the learned warm start; and the CPU oracle's full
solves on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 128
S = 4
RTOL = 1e-8
SEED = 0
MAXIT = 20000


def algorithmic_bytes(n, nnz, s=S):
    """Bytes one launch of each kernel class must move (FP64 values and
    vectors, int32 indices).  The 7-point matrix has a constant diagonal, so
    the Jacobi scaling is one constant c: no Z column of the block is stored,
    each reader forms c * r or c * AZ(:,j-1) itself.
      matrix power j < s: val + colind (12 nnz) + rowptr (4 n) + gathered input, AZ_j (16 n)
      last power + moments: 12 nnz + 4 n + input, AZ_s, r (24 n) + AZ_1..AZ_{s-2} (8 (s-2) n)
      block update: reads AZ, P_old, AP_old, x, r (8 (3s + 2) n),
                    writes P, AP, x, r (8 (2s + 2) n)
      Chebyshev basis, block Gram pass: reads Z, AZ, AP_old, r (8 (3s + 1) n)
    """
    return {
        "mpk": 12 * nnz + 4 * n + 16 * n,
        "mpk_last": 12 * nnz + 4 * n + 24 * n + 8 * (s - 2) * n,
        "update": 8 * (3 * s + 2) * n + 8 * (2 * s + 2) * n,
        "gram": 8 * (3 * s + 1) * n,
    }


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("common.hpp", "operators.hpp", "kernels.hpp", "small_solve.hpp", "gram.hpp",
              "engine.hpp", "setup_kernels.hpp", "capi.hip", "temporal.hpp", "amg.hip"):
        with open(os.path.join(ROOT, "paper_2501_03743_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(name, sha, key="fetch_write_bytes_per_launch"):
    """Bytes moved between the L2 caches and memory (FETCH_SIZE + WRITE_SIZE
    counters, scaled by the copy calibration) per launch of a kernel, from a
    committed rocprofv3 counter summary, if it was taken on the current
    kernel sources; None otherwise."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != sha:
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def median_time(fn, reps=5):
    """Median wall time of `reps` runs after one warm-up (each run synchronised)."""
    import torch
    fn()
    ts, out = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts)), out


def oracle_threads():
    import oracle
    return oracle.set_threads(0)


def cpu_baseline(budget_one_thread_s=40.0):
    """The oracle (plain C, FP64, OpenMP over fixed row chunks) on the same
    128^3 CSR problem, run to the end: the s-step solve (s = 4) with all host
    threads (the value), the same with one thread, and standard PCG with all
    threads.  The one-thread solve is skipped if a probe of two outer
    iterations predicts more than `budget_one_thread_s`."""
    import oracle
    from paper_2501_03743_amd import workloads as wl
    csr = wl.stencil_csr("3d7", (N, N, N))
    op = oracle.Operator("csr", csr=csr)
    b = wl.normal_rhs(N ** 3, SEED)
    cores = oracle_threads()
    t0 = time.perf_counter()
    r = oracle.sstep(op, b, S, rtol=RTOL, maxit=MAXIT)
    t_all = time.perf_counter() - t0
    t0 = time.perf_counter()
    rp = oracle.pcg(op, b, rtol=RTOL, maxit=MAXIT)
    t_pcg = time.perf_counter() - t0
    oracle.set_threads(1)
    t_one = None
    try:
        t0 = time.perf_counter()
        oracle.sstep(op, b, S, fixed_outer=2)
        per = (time.perf_counter() - t0) / 2
        if per * r.outer <= budget_one_thread_s:
            t0 = time.perf_counter()
            r1 = oracle.sstep(op, b, S, rtol=RTOL, maxit=MAXIT)
            t_one = time.perf_counter() - t0
            assert r1.outer == r.outer
        else:
            t_one = None
    finally:
        oracle.set_threads(cores)
    return {"value": t_all, "unit": "s", "cores": cores, "kind": "oracle",
            "sample": "the full 128^3 CSR s-step solve (s=4, rtol 1e-8, %d outer iterations) with "
                      "%d OpenMP threads" % (r.outer, cores),
            "one_thread_s": t_one, "pcg_all_threads_s": t_pcg, "pcg_iterations": rp.outer,
            "outer": r.outer, "true_rel": r.true_rel}


def oracle_small(csr0, b0):
    """The oracle on the launch-bound 2D 64^2 problem: s-step (s = 4 and 1)
    and standard PCG, one thread and all threads."""
    import oracle
    op = oracle.Operator("csr", csr=csr0)
    cores = oracle_threads()
    out = {"cores": cores}
    for threads, tag in ((1, "one_thread"), (cores, "all_threads")):
        oracle.set_threads(threads)
        for name, fn in (("sstep_s4", lambda: oracle.sstep(op, b0, 4, rtol=RTOL)),
                         ("sstep_s1", lambda: oracle.sstep(op, b0, 1, rtol=RTOL)),
                         ("pcg", lambda: oracle.pcg(op, b0, rtol=RTOL))):
            fn()
            t0 = time.perf_counter()
            for _ in range(5):
                rr = fn()
            out["%s_%s_ms" % (name, tag)] = 1e3 * (time.perf_counter() - t0) / 5
            out["%s_iterations" % name] = rr.outer
    oracle.set_threads(cores)
    return out


def bench_batch(H, count=32, lo=32, hi=160, seed=0):
    """`count` variable-coefficient 7-point systems, sides L ~ U{lo..hi}, k =
    exp(g) with g a Gaussian random field (sigma 0.5, correlation length 0.1),
    b ~ N(0, 1): one batched solve (autotuned schedule, tiles and grid)
    against the same systems solved one after another, all to rtol 1e-8 with
    FP32 matrix powers and FP64 moments, s x s solves and refinement."""
    import torch
    from paper_2501_03743_amd import workloads as wl
    sides = [int(v) for v in wl.batch_sides(seed, count, lo, hi)]
    mats, bs, keep = [], [], []
    for i, L in enumerate(sides):
        shape = (L, L, L)
        k = torch.exp(wl.gaussian_random_field_device(shape, 0.5, 0.1, 1000 + i))
        mats.append(H.matrix_stencil("3d7_vark", shape, k=k))
        bs.append(torch.from_numpy(wl.normal_rhs(L ** 3, 2000 + i)).cuda())
        keep.append(k)
    torch.cuda.synchronize()
    t = time.perf_counter()
    tune = H.autotune_batch(mats, bs, s=S)
    tune_s = time.perf_counter() - t
    xs = [torch.zeros_like(b) for b in bs]

    def batch_once():
        for v in xs:
            v.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st, it, tr = H.solve_batch(mats, bs, xs, s=S, rtol=RTOL, maxit=MAXIT, tune=tune)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st, it, tr

    batch_once()
    reps = [batch_once() for _ in range(3)]
    t_batch = float(np.median([r[0] for r in reps]))
    _, st, it, tr = reps[-1]
    from paper_2501_03743_amd import sstep
    forms = {}
    for name, tn in (("persistent", sstep.Tune(tile_rows=tune.tile_rows, grid=tune.grid or 1024,
                                               order=tune.order, schedule=0)),
                     ("persistent_run4", sstep.Tune(tile_rows=tune.tile_rows,
                                                    grid=tune.grid or 1024, order=tune.order,
                                                    schedule=0, run=4)),
                     ("stepped", sstep.Tune(tile_rows=tune.tile_rows, schedule=1))):
        ts = []
        for _ in range(3):
            for v in xs:
                v.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rcn, stn, _, trn = H.solve_batch(mats, bs, xs, s=S, rtol=RTOL, maxit=MAXIT, tune=tn)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        forms[name] = {"s": float(np.median(ts)), "all_converged": bool((stn == 0).all()),
                       "max_true_rel": float(np.max(trn))}

    def seq_once(precision):
        res = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for M, b, v in zip(mats, bs, xs):
            v.zero_()
            res.append(H.solve(M, b, v, s=S, rtol=RTOL, maxit=MAXIT, precision=precision))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, res

    seq_once("mixed_ir")
    runs = [seq_once("mixed_ir") for _ in range(3)]
    t_seq = float(np.median([r[0] for r in runs]))
    res_seq = runs[-1][1]
    t_seq64, res64 = seq_once("fp64")
    out = {
        "workload": "%d x 3D 7-point variable-coefficient Poisson, L ~ U{%d..%d} (sum n = %d), "
                    "k = exp(GRF sigma 0.5, l 0.1), b ~ N(0,1), s=4, rtol 1e-8"
                    % (count, lo, hi, sum(L ** 3 for L in sides)),
        "sides": sides,
        "tune": tune.as_dict(), "autotune_s": tune_s,
        "batch_s": t_batch,
        "persistent_launch_s": forms["persistent"]["s"],
        "stepped_s": forms["stepped"]["s"],
        "forms": forms,
        "sequential_mixed_s": t_seq,
        "sequential_fp64_s": t_seq64,
        "speedup_vs_sequential_mixed": t_seq / t_batch,
        "timing": "median of 3 runs each, wall time around the call",
        "all_converged": bool((st == 0).all()) and all(r.status == 0 for r in res_seq),
        "max_true_rel_batch": float(np.max(tr)),
        "max_true_rel_sequential": float(max(r.true_rel for r in res_seq)),
    }
    for M in mats:
        M.close()
    return out


def bench_net_steps(H, steps, side=96, batch=4):
    """Training steps and batch-1 forwards of the warm-start network on random
    inputs (timing and counter target; the values are irrelevant here)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    net = H.net((side, side, side), max_batch=batch, seed=0)
    inp = torch.randn((batch, side, side, side, 2), generator=g, device="cuda")
    tgt = torch.randn((batch, side, side, side), generator=g, device="cuda")
    y = torch.empty_like(tgt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.forward(inp, y)
        _, dy = net.loss_h1(y, tgt, 1e-3)
        net.zero_grad()
        net.backward(dy)
        net.adam_step(1e-3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    one = inp[:1].contiguous()
    for _ in range(steps):
        net.forward(one)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # the inference call of the warm start (features, forward, FP64 output)
    n = side ** 3
    logk = torch.randn(n, generator=g, device="cuda", dtype=torch.float64)
    f = torch.randn(n, generator=g, device="cuda", dtype=torch.float64)
    x0 = torch.empty_like(f)
    for _ in range(steps):
        net.predict(logk, f, 1.0, out=x0)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    net.close()
    return {"side": side, "batch": batch, "steps": steps,
            "train_step_ms": 1e3 * (t1 - t0) / steps, "forward_batch1_ms": 1e3 * (t2 - t1) / steps,
            "predict_ms": 1e3 * (t3 - t2) / steps}


def bench_paper_1e9(H):
    """Sec. V-B's weak-scaled problem (64 x 250^3 = 10^9 unknowns, 2101
    iterations for PFCG and PCGs with s = 1 on 64 GPUs) on one GPU, as the
    1000^3 cube in stencil form: time to solution of each method, one run
    each (the solves take seconds, the set-up is excluded)."""
    import torch
    N = 1000
    A = H.matrix_stencil("3d7", (N, N, N))
    A.set_preconditioner("none")
    b = torch.ones(N ** 3, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    out = {"workload": "3D 7-point 1000^3 stencil (n=10^9), b=1, no preconditioner, rtol 1e-6",
           "paper_iterations_64_gpus": 2101}
    for name, kw in (("pfcg", {"method": "pfcg"}), ("pcg", {"method": "pcg"}),
                     ("sstep_s4", {"s": 4}), ("sstep_s4_mixed_ir", {"s": 4, "precision": "mixed_ir",
                                                                  "inner_rtol": 1e-3})):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = H.solve(A, b, x, rtol=1e-6, maxit=8000, **kw)
        torch.cuda.synchronize()
        out[name] = {"tts_s": time.perf_counter() - t0, "status": r.status, "outer": r.outer,
                     "cg_equiv": r.cg_equiv, "true_rel": r.true_rel}
        print("[paper-1e9] %s %s" % (name, json.dumps(out[name])), file=sys.stderr, flush=True)
    A.close()
    return out


def bench_warmstart(H, n_train=2000, n_eval=200, side=96, epochs=40, lr=2e-3, batch=4,
                    log=None, sweeps=16, n_loose=50, n_forms=20):
    """The learned warm start on -div(k grad u) = f at side^3: log k a Gaussian
    random field (sigma 1, correlation length 0.1), f a random sum of 16
    Fourier modes; the network trained on n_train solver solutions (seeds
    10000..), evaluated on n_eval held-out seeds (20000..) against x0 = 0, and
    the mixed-precision + warm-start form against plain FP64 s-step and
    standard CG at the same tolerance."""
    import torch
    from paper_2501_03743_amd import warmstart as ws
    from paper_2501_03743_amd import workloads as wl
    shape = (side, side, side)
    t0 = time.time()
    data = ws.generate(H, shape, list(range(10000, 10000 + n_train)), s=S, rtol=RTOL, log=log)
    gen_s = time.time() - t0
    model = ws.WarmStart(H, shape, batch=batch, seed=0)
    t0 = time.time()
    hist = model.fit(data, epochs, lr=lr, log=log)
    train_s = time.time() - t0
    del data
    torch.cuda.empty_cache()
    seeds = list(range(20000, 20000 + n_eval))
    rec = ws.evaluate(H, model, seeds, s=S, rtol=RTOL, sweeps=sweeps)
    summ = ws.summarize(rec)
    # the same held-out seeds at a looser tolerance, where a guess's share of
    # the decades CG must gain is larger
    summ_1e6 = ws.summarize(ws.evaluate(H, model, seeds[:n_loose], s=S, rtol=1e-6, sweeps=sweeps))
    # the full forms at equal final accuracy on the first held-out seeds
    forms = {}
    m = min(n_forms, n_eval)
    for name, kw, warm in (("pcg_fp64_x0_0", {"method": "pcg"}, False),
                           ("sstep_fp64_x0_0", {}, False),
                           ("sstep_mixed_x0_0", {"precision": "mixed_ir"}, False),
                           ("sstep_mixed_warm", {"precision": "mixed_ir"}, True)):
        ts, its, trs = [], [], []
        for seed in seeds[:m]:
            logk, k, f, b = wl.warm_start_problem(shape, seed)
            A = H.matrix_stencil("3d7_vark", shape, k=k)
            x = torch.zeros_like(b)
            if kw.get("precision"):
                H.solve(A, b, x, s=S, rtol=RTOL, **kw)   # FP32 copy built outside the timing
                x.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if warm:
                model.predict(logk, f, out=x)
            r = H.solve(A, b, x, s=S, rtol=RTOL, maxit=MAXIT, warm_start=warm,
                        warm_sweeps=sweeps if warm else 0, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
            its.append(r.cg_equiv if kw.get("method") != "pcg" else r.outer)
            trs.append(r.true_rel)
            A.close()
        forms[name] = {"mean_s": float(np.mean(ts)), "mean_cg_steps": float(np.mean(its)),
                       "max_true_rel": float(np.max(trs))}
    params = model.net.count
    model.close()
    return {
        "workload": "-div(k grad u)=f on %d^3, log k GRF (sigma 1, l 0.1), f = 16 Fourier modes, "
                    "s=4, rtol 1e-8" % side,
        "train_samples": n_train, "eval_samples": n_eval, "epochs": len(hist),
        "loss": "energy e^T (L + 1e-3 I) e", "smoothing_sweeps": sweeps,
        "generate_s": gen_s, "train_s": train_s, "loss_first": hist[0], "loss_last": hist[-1],
        "params": params,
        "held_out": summ, "held_out_rtol_1e-6_first_%d" % n_loose: summ_1e6,
        "forms_first_%d" % m: forms,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-27pt", action="store_true",
                    help="skip the 256^3 27-point FP64 / mixed-precision comparison")
    ap.add_argument("--skip-oracle-27pt", action="store_true",
                    help="skip the oracle's 256^3 27-point reference solve")
    ap.add_argument("--skip-batch", action="store_true", help="skip the batched solves")
    ap.add_argument("--skip-warmstart", action="store_true",
                    help="skip the bounded learned-warm-start run")
    ap.add_argument("--only-timed", action="store_true",
                    help="only the timed solves (for profiler runs)")
    ap.add_argument("--warmstart", action="store_true",
                    help="only the learned warm start at its full budget (several minutes)")
    ap.add_argument("--ws-train", type=int, default=2000)
    ap.add_argument("--ws-eval", type=int, default=200)
    ap.add_argument("--ws-side", type=int, default=96)
    ap.add_argument("--ws-epochs", type=int, default=40)
    ap.add_argument("--csr256-outer", type=int, default=0,
                    help="only the 256^3 7-point CSR solve for this many outer iterations "
                         "(s = 4, no stopping test): a short target for counter runs")
    ap.add_argument("--csr256-basis", default="monomial",
                    help="basis of the --csr256-outer run (monomial or chebyshev)")
    ap.add_argument("--csr27-outer", type=int, default=0,
                    help="only the 27-point 256^3 CSR solve for this many outer iterations "
                         "(s = 4, FP64, no stopping test): a short target for counter runs")
    ap.add_argument("--paper-1e9", action="store_true",
                    help="only the paper's largest problem on one GPU: 3D 7-point 1000^3 "
                         "(10^9 unknowns, stencil form), b = 1, no preconditioner, rtol 1e-6; "
                         "PFCG, standard PCG and the s-step form (about 3 minutes)")
    ap.add_argument("--net-steps", type=int, default=0,
                    help="only this many training steps of the warm-start network at 96^3, "
                         "batch 4 (forward, energy loss, backward, Adam) and as many batch-1 "
                         "forwards: a short target for kernel-trace and MFMA counter runs")
    ap.add_argument("--stencil-outer", type=int, default=0,
                    help="only the 3D 7-point matrix-free solve (--stencil-side, s = 4, "
                         "FP64) for this many outer iterations, with the temporally blocked "
                         "powers (--stencil-form tb) or one launch per power (per-power): a "
                         "short target for kernel-trace and counter runs")
    ap.add_argument("--stencil-side", type=int, default=128)
    ap.add_argument("--stencil-form", default="tb", choices=("tb", "per-power"))
    ap.add_argument("--amg-solves", type=int, default=0,
                    help="only this many AMG-preconditioned s-step solves of the 3D 7-point "
                         "128^3 CSR system (s = 4, rtol 1e-8): a short target for kernel-trace "
                         "runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only the library's plain copy of 1 GiB, three times (the "
                         "reference for the FETCH_SIZE / WRITE_SIZE counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the solver has no sharding or "
              "collectives); --gpus %d is not supported, use --gpus 1" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2501_03743_amd import sstep
    from paper_2501_03743_amd import workloads as wl

    def log(m):
        print("[bench] " + m, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    H = sstep.Handle(0)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        ms = H.stream_probe(src, dst, reps=3)
        print(json.dumps({"copy_bytes": src.numel() * 8, "copies": 4, "ms_per_copy": ms}))
        return
    if args.net_steps > 0:
        print(json.dumps({"net_steps": bench_net_steps(H, args.net_steps)}))
        return
    if args.paper_1e9:
        print(json.dumps({"paper_1e9": bench_paper_1e9(H)}))
        return
    if args.csr256_outer > 0:
        N3 = 256
        A3 = H.matrix_csr_from_stencil("3d7", (N3, N3, N3))
        b3 = torch.from_numpy(wl.normal_rhs(N3 ** 3, SEED)).cuda()
        x3 = torch.zeros_like(b3)
        r3 = H.solve(A3, b3, x3, s=S, fixed_outer=args.csr256_outer, profile=True,
                     basis=args.csr256_basis)
        print(json.dumps({"workload": "3D 7-point 256^3 CSR", "csr_form": A3.csr_form,
                          "basis": args.csr256_basis, "nnz": A3.nnz, "outer": r3.outer,
                          "profile": r3.profile}))
        return
    if args.stencil_outer > 0:
        Ns = args.stencil_side
        os.environ["SSP_MPK_TEMPORAL"] = "2" if args.stencil_form == "tb" else "0"
        As = H.matrix_stencil("3d7", (Ns, Ns, Ns))
        os.environ.pop("SSP_MPK_TEMPORAL")
        bs = torch.from_numpy(wl.normal_rhs(Ns ** 3, SEED)).cuda()
        xs = torch.zeros_like(bs)
        for _ in range(3):
            xs.zero_()
            rs = H.solve(As, bs, xs, s=S, fixed_outer=args.stencil_outer, profile=True)
        print(json.dumps({"workload": "3D 7-point %d^3 matrix-free" % Ns,
                          "form": args.stencil_form, "outer": rs.outer, "profile": rs.profile}))
        return
    if args.amg_solves > 0:
        Aa = H.matrix_csr_from_stencil("3d7", (N, N, N))
        H.set_amg(Aa)
        ba = torch.from_numpy(wl.normal_rhs(N ** 3, SEED)).cuda()
        xa = torch.zeros_like(ba)
        for _ in range(args.amg_solves):
            xa.zero_()
            ra = H.solve(Aa, ba, xa, s=S, rtol=RTOL, maxit=MAXIT)
        print(json.dumps({"workload": "3D 7-point 128^3 CSR, AMG", "levels": H.amg_levels(Aa),
                          "outer": ra.outer, "true_rel": ra.true_rel}))
        return
    if args.csr27_outer > 0:
        N2 = 256
        A2 = H.matrix_csr_from_stencil("3d27", (N2, N2, N2))
        b2 = torch.from_numpy(wl.normal_rhs(N2 ** 3, SEED)).cuda()
        x2 = torch.zeros_like(b2)
        r2 = H.solve(A2, b2, x2, s=S, fixed_outer=args.csr27_outer, profile=True)
        print(json.dumps({"workload": "3D 27-point 256^3 CSR", "csr_form": A2.csr_form,
                          "nnz": A2.nnz, "outer": r2.outer, "profile": r2.profile}))
        return
    if args.warmstart:
        print(json.dumps({"config_warm_start": bench_warmstart(
            H, args.ws_train, args.ws_eval, args.ws_side, args.ws_epochs,
            log=lambda m: log("warmstart: " + m))}))
        return
    n = N ** 3
    A = H.matrix_csr_from_stencil("3d7", (N, N, N))
    b = torch.from_numpy(wl.normal_rhs(n, SEED)).cuda()
    x = torch.zeros_like(b)
    torch.cuda.synchronize()

    def solve(profile=False, **kw):
        x.zero_()
        return H.solve(A, b, x, s=kw.pop("s", S), rtol=RTOL, maxit=MAXIT, profile=profile, **kw)

    for _ in range(args.warmup):
        res = solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = solve()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tts = elapsed / args.steps
    if res.status != 0:
        print("bench.py: solve did not converge (status %d)" % res.status, file=sys.stderr)
        sys.exit(1)
    if args.only_timed:
        print(json.dumps({"tts_s": tts, "outer": res.outer}))
        return
    log("headline: %.2f ms per solve, %d outer iterations" % (1e3 * tts, res.outer))

    # kernel durations from HIP events on the library's stream (same solves, profiled)
    def profile_means(fn, reps):
        ms = np.zeros(sstep.PROFILE_CLASSES)
        cnt = np.zeros(sstep.PROFILE_CLASSES)
        for _ in range(reps):
            r = fn()
            ms += np.array(r.profile["ms"])
            cnt += np.array(r.profile["launches"])
        return ms / np.maximum(cnt, 1), cnt / reps, ms / reps

    mean_ms, launches, per_solve_ms = profile_means(lambda: solve(profile=True), args.steps)
    nnz = A.nnz
    ab = algorithmic_bytes(n, nnz)
    achieved = ab["mpk"] / (mean_ms[0] * 1e-3) / 1e9
    sha = kernel_source_sha()
    traffic = read_traffic("traffic_csr_mpk_3d7_128.txt", sha)

    # achievable bandwidth: the library's own streaming read and copy of 1 GiB
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    read_gbs = src.numel() * 8 / (H.stream_probe(src, reps=10) * 1e-3) / 1e9
    copy_gbs = 2 * src.numel() * 8 / (H.stream_probe(src, dst, reps=10) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    log("stream probe: read %.0f GB/s, copy %.0f GB/s" % (read_gbs, copy_gbs))

    # matrix powers at 256^3 (the 1.4 GB sliced-ELL matrix does not fit the 256 MB
    # memory-side cache): per-launch rates over 10 profiled outer iterations
    N3 = 256
    n3 = N3 ** 3
    A3 = H.matrix_csr_from_stencil("3d7", (N3, N3, N3))
    b3 = torch.from_numpy(wl.normal_rhs(n3, SEED)).cuda()
    x3 = torch.zeros_like(b3)
    H.solve(A3, b3, x3, s=S, fixed_outer=2)
    x3.zero_()
    r3 = H.solve(A3, b3, x3, s=S, fixed_outer=10, profile=True)
    ab3 = algorithmic_bytes(n3, A3.nnz)
    m3 = np.array(r3.profile["ms"]) / np.maximum(np.array(r3.profile["launches"]), 1)
    mpk3_gbs = ab3["mpk"] / (m3[0] * 1e-3) / 1e9
    big = {"workload": "3D 7-point 256^3 CSR (n=16777216, nnz=%d), s=4, 10 outer iterations"
                       % A3.nnz,
           "mpk_gbs": mpk3_gbs, "mpk_frac_of_peak": mpk3_gbs / HBM_PEAK_GBS,
           "mpk_last_gbs": ab3["mpk_last"] / (m3[1] * 1e-3) / 1e9,
           "update_gbs": ab3["update"] / (m3[2] * 1e-3) / 1e9,
           "mpk_mean_launch_ms": m3[0]}
    big["gram_traffic"] = read_traffic("gram_mfma_3d7_256_chebyshev.txt", sha,
                                       key="gram_fetch_write_bytes_per_launch")
    # the Chebyshev basis at 256^3: the block Gram pass on the FP64 matrix cores
    cheb_gram = {}
    for sc in (4, 8):
        x3.zero_()
        rc3 = H.solve(A3, b3, x3, s=sc, fixed_outer=6, profile=True, basis="chebyshev")
        mc = np.array(rc3.profile["ms"]) / np.maximum(np.array(rc3.profile["launches"]), 1)
        gb = algorithmic_bytes(n3, A3.nnz, sc)["gram"]
        cheb_gram["s%d" % sc] = {"gram_ms": mc[4], "gram_bytes": gb,
                                 "gram_gbs": gb / (mc[4] * 1e-3) / 1e9,
                                 "gram_frac_of_peak": gb / (mc[4] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "gram_fp64_flops": 2 * sc * (2 * sc + 1) * n3}
    big["chebyshev_gram_pass"] = cheb_gram
    A3.close()
    del b3, x3
    torch.cuda.empty_cache()
    log("256^3 matrix power %.0f GB/s" % mpk3_gbs)

    # comparisons at 128^3 (outside the timed region; medians of 5 solves)
    compare = {}

    def row(fn):
        t, r = median_time(fn)
        return {"tts_s": t, "outer": r.outer, "cg_equiv": r.cg_equiv, "status": r.status,
                "true_rel": r.true_rel, "restarts": r.restarts}

    compare["pcg_csr"] = row(lambda: solve(method="pcg"))
    compare["pfcg_csr"] = row(lambda: solve(method="pfcg"))
    compare["sstep_mixed_ir_csr"] = row(lambda: solve(precision="mixed_ir"))
    per_s = {}
    for sv in (1, 2, 4, 8):
        per_s[str(sv)] = row(lambda: solve(s=sv))
    per_s["8_restarts"] = row(lambda: solve(s=8, restarts=3))
    compare["sstep_csr_by_s"] = per_s
    cheb = {}
    for sv in (4, 8, 12, 16):
        cheb[str(sv)] = row(lambda: solve(s=sv, basis="chebyshev"))
    cheb["8_mixed_ir"] = row(lambda: solve(s=8, basis="chebyshev", precision="mixed_ir"))
    compare["sstep_csr_chebyshev_by_s"] = cheb
    # the AMG preconditioner (smoothed aggregation; B^-1 = one weighted-Jacobi
    # V-cycle) on a CSR copy of the same operator; its one-time host setup is
    # timed on its own and is not part of the solve times
    Aa = H.matrix_csr_from_stencil("3d7", (N, N, N))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H.set_amg(Aa)
    torch.cuda.synchronize()
    amg_rows = {"setup_s": time.perf_counter() - t0, "levels": H.amg_levels(Aa)}

    def solve_amg(**kw):
        x.zero_()
        return H.solve(Aa, b, x, rtol=RTOL, maxit=MAXIT, **kw)

    for sv in (1, 2, 4, 8):
        amg_rows[str(sv)] = row(lambda: solve_amg(s=sv))
    compare["sstep_csr_amg_by_s"] = amg_rows
    Aa.close()
    log("AMG s=4: %.2f ms, %d outer" % (amg_rows["4"]["tts_s"] * 1e3, amg_rows["4"]["outer"]))
    As = H.matrix_stencil("3d7", (N, N, N))

    def solve_st(**kw):
        x.zero_()
        return H.solve(As, b, x, rtol=RTOL, maxit=MAXIT, **kw)

    st_s = {}
    for sv in (1, 2, 4, 8):
        st_s[str(sv)] = row(lambda: solve_st(s=sv))
    st_s["8_chebyshev"] = row(lambda: solve_st(s=8, basis="chebyshev"))
    st_s["4_mixed_ir"] = row(lambda: solve_st(s=4, precision="mixed_ir"))
    compare["sstep_stencil_by_s"] = st_s
    compare["pcg_stencil"] = row(lambda: solve_st(method="pcg"))
    compare["pfcg_stencil"] = row(lambda: solve_st(method="pfcg"))

    # plain SpMV per operator form / CSR kernel variant (HIP events on the same stream)
    def spmv_ms(M, reps=20):
        y = torch.empty_like(b)
        H.spmv(M, b, y)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            H.spmv(M, b, y)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    spmv = {"csr_autotuned_ms": spmv_ms(A), "csr_form": A.csr_form, "stencil_ms": spmv_ms(As)}
    saved = os.environ.get("SSP_CSR_VARIANT")
    for v, name in ((0, "csr_staged_ms"), (1, "csr_row_ms"), (2, "csr_sell_ms")):
        os.environ["SSP_CSR_VARIANT"] = str(v)
        Mv = H.matrix_csr_from_stencil("3d7", (N, N, N))
        spmv[name] = spmv_ms(Mv)
        Mv.close()
    if saved is None:
        del os.environ["SSP_CSR_VARIANT"]
    else:
        os.environ["SSP_CSR_VARIANT"] = saved
    plain_bytes = 12 * nnz + 4 * n + 16 * n
    spmv["csr_plain_bytes"] = plain_bytes
    spmv["csr_best_gbs"] = plain_bytes / (min(spmv["csr_staged_ms"], spmv["csr_row_ms"],
                                              spmv["csr_sell_ms"]) * 1e-3) / 1e9
    spmv["stencil_gbs"] = 16 * n / (spmv["stencil_ms"] * 1e-3) / 1e9
    compare["spmv"] = spmv
    As.close()
    log("128^3 comparisons done")

    # 2D 5-point 64^2 (everything cache-resident, launch-bound): x* ~ U(-1,1)
    # from seeds 0..4, b = A x*; medians of 5 solves per form
    small = []
    csr0 = wl.stencil_csr("2d5", (64, 64))
    A0 = H.matrix_csr(*[torch.from_numpy(a).cuda() for a in csr0], flags=sstep.COPY)
    b0_seed0 = None
    for seed in range(5):
        b0h = wl.csr_matvec(csr0, wl.uniform_solution(64 * 64, seed))
        if seed == 0:
            b0_seed0 = b0h
        b0 = torch.from_numpy(b0h).cuda()
        rw = {"seed": seed}
        x0 = torch.zeros_like(b0)
        for name, kw in (("sstep_s4", {"s": 4}), ("sstep_s1", {"s": 1}), ("pcg", {"method": "pcg"}),
                         ("pfcg", {"method": "pfcg"})):
            def one(kw=kw):
                x0.zero_()
                return H.solve(A0, b0, x0, rtol=RTOL, **kw)
            t, rr = median_time(one)
            rw[name + "_ms"] = 1e3 * t
            rw[name + "_iterations"] = rr.cg_equiv if name.startswith("sstep") else rr.outer
        small.append(rw)
    A0.close()
    config0 = {"workload": "2D 5-point 64^2 (n=4096), CSR, Jacobi, x* ~ U(-1,1) seeds 0..4, "
                           "b = A x*, rtol 1e-8", "rows": small}
    if not args.no_cpu_baseline:
        config0["oracle_seed0"] = oracle_small(csr0, b0_seed0)

    # 3D 27-point 256^3 (n = 16.8M, 449M stored entries), Jacobi, s = 4, to rtol 1e-10:
    # plain FP64 s-step and standard CG versus the FP32-inner / FP64-refinement form,
    # CSR and matrix-free; each x compared with the oracle's FP64 solution
    # (27-point stencil form, all host threads, rtol 1e-10)
    config2 = None
    if not args.skip_27pt:
        N2 = 256
        n2 = N2 ** 3
        b2h = wl.normal_rhs(n2, SEED)
        b2 = torch.from_numpy(b2h).cuda()
        x2 = torch.zeros_like(b2)
        xo = None
        config2 = {"workload": "3D 27-point 256^3 (n=16777216), Jacobi, s=4, b~N(0,1) seed 0, "
                               "rtol 1e-10", "reference": None}
        if not args.skip_oracle_27pt:
            import oracle
            t0 = time.perf_counter()
            ro = oracle.sstep(oracle.Operator("3d27", (N2, N2, N2)), b2h, S, rtol=1e-10,
                              maxit=MAXIT)
            config2["reference"] = {"kind": "oracle", "form": "27-point stencil", "s": S,
                                    "rtol": 1e-10, "outer": ro.outer, "status": ro.status,
                                    "true_rel": ro.true_rel, "host_s": time.perf_counter() - t0,
                                    "threads": oracle_threads()}
            xo = torch.from_numpy(ro.x).cuda()
            del ro
            log("27-point oracle reference: %.1f s" % config2["reference"]["host_s"])

        def run2(M, **kw):
            x2.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            rr = H.solve(M, b2, x2, rtol=1e-10, maxit=MAXIT, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            out = {"tts_s": dt, "status": rr.status, "outer": rr.outer,
                   "true_rel": rr.true_rel}
            if kw.get("precision") == "mixed_ir":
                out["refinements"] = len(rr.hist) - 1
            if xo is not None:
                out["rel_err_vs_oracle"] = float(torch.linalg.vector_norm(x2 - xo) /
                                                 torch.linalg.vector_norm(xo))
            return out

        A2 = H.matrix_csr_from_stencil("3d27", (N2, N2, N2))
        config2["nnz"] = A2.nnz
        # matrix powers of the 27-point matrix (5.4 GB, streamed from HBM):
        # per-launch rates over 4 profiled outer iterations
        x2.zero_()
        rp = H.solve(A2, b2, x2, s=S, fixed_outer=4, profile=True)
        mp = np.array(rp.profile["ms"]) / np.maximum(np.array(rp.profile["launches"]), 1)
        ab2 = algorithmic_bytes(n2, A2.nnz)
        config2["roofline_mpk"] = {
            "bound": "hbm", "achieved": ab2["mpk"] / (mp[0] * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": ab2["mpk"] / (mp[0] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "traffic": read_traffic("traffic_csr_3d27_256.txt", kernel_source_sha()),
            "kernel": "matrix-powers CSR SpMV + Jacobi (power j < s), 27-point 256^3",
            "bytes_per_launch": ab2["mpk"], "mean_launch_ms": mp[0]}
        run2(A2, s=S, precision="mixed_ir")   # first use builds the FP32 copy
        config2["csr_sstep_fp64"] = run2(A2, s=S)
        config2["csr_sstep_mixed_ir"] = run2(A2, s=S, precision="mixed_ir")
        config2["csr_sstep_mixed_ir_inner1e-6"] = run2(A2, s=S, precision="mixed_ir",
                                                       inner_rtol=1e-6)
        config2["csr_pcg_fp64"] = run2(A2, method="pcg")
        A2.close()
        torch.cuda.empty_cache()
        # the same operator matrix-free (nothing stored but the two coefficients)
        A2 = H.matrix_stencil("3d27", (N2, N2, N2))
        run2(A2, s=S, precision="mixed_ir")
        config2["stencil_sstep_fp64"] = run2(A2, s=S)
        config2["stencil_sstep_mixed_ir"] = run2(A2, s=S, precision="mixed_ir")
        config2["stencil_pcg_fp64"] = run2(A2, method="pcg")
        A2.close()
        del b2, x2, xo
        torch.cuda.empty_cache()
        log("27-point 256^3 done")

    config3 = None
    if not args.skip_batch:
        config3 = {"batch32_L32_160": bench_batch(H),
                   "batch128_L12_40": bench_batch(H, count=128, lo=12, hi=40, seed=1)}
        log("batches done")

    config4 = None
    if not args.skip_warmstart:
        # bounded: 1500 training solutions, 24 epochs, 50 held-out seeds
        config4 = bench_warmstart(H, n_train=1500, n_eval=50, epochs=24, n_loose=20, n_forms=20,
                                  log=lambda m: log("warmstart: " + m))
        config4["budget"] = "bounded: 1500 training solutions, 24 epochs, 50 held-out seeds"
        log("warm start done")

    out = {
        "metric": "time-to-solution @rtol 1e-8 (s) + SpMV/matrix-powers HBM GB/s, s-step vs CG",
        "value": tts,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tts * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D 7-point Poisson 128^3 (n=2097152, nnz=%d), FP64 CSR, Jacobi, "
                               "s=4, b~N(0,1) seed 0, x0=0, rtol 1e-8" % nnz,
                   "method": "preconditioned s-step CG (Chronopoulos-Gear), s=4",
                   "csr_kernel_form": A.csr_form, "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "matrix-powers CSR SpMV + Jacobi (power j < s)",
                     "note": "the 176 MB sliced-ELL matrix stays in the 256 MB memory-side "
                             "cache at 128^3; roofline_hbm_resident is the same kernel at "
                             "256^3, streamed from HBM",
                     "bytes_per_launch": ab["mpk"], "mean_launch_ms": mean_ms[0]},
        "roofline_hbm_resident": {
            "bound": "hbm", "achieved": mpk3_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": mpk3_gbs / HBM_PEAK_GBS,
            "traffic": read_traffic("traffic_csr_mpk_3d7_256.txt", sha),
            "kernel": "matrix-powers CSR SpMV + Jacobi (power j < s), 3D 7-point 256^3",
            "bytes_per_launch": ab3["mpk"], "mean_launch_ms": m3[0]},
        "achievable": {"stream_read_gbs": read_gbs, "stream_copy_gbs": copy_gbs,
                       "mpk_frac_of_read": achieved / read_gbs,
                       "mpk256_frac_of_read": mpk3_gbs / read_gbs,
                       "kernels": "libsstep k_stream_read / k_stream_copy, 1 GiB"},
        "iterations": {"outer": res.outer, "cg_equiv": res.cg_equiv, "true_rel": res.true_rel},
        "kernels": {
            "mpk_gbs": achieved,
            "mpk_last_gram_solve_ms": mean_ms[1],
            "mpk_last_gbs": ab["mpk_last"] / (mean_ms[1] * 1e-3) / 1e9,
            "update_ms": mean_ms[2],
            "update_gbs": ab["update"] / (mean_ms[2] * 1e-3) / 1e9,
            "kernel_ms_per_solve": per_solve_ms.tolist(),
            "launches_per_solve": launches.tolist(),
            "kernel_source_sha": sha,
        },
        "compare": compare,
        "csr_3d7_256": big,
        "config_2d5_64": config0,
        "config_27pt_256_mixed": config2,
        "config_batch32": config3,
        "config_warm_start": config4,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        log("cpu baseline: %.2f s" % out["cpu_baseline"]["value"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
