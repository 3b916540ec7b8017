"""Throughput of MgNet-preconditioned flexible GMRES on one MI355X.

Workload: 128x128 cells, 32 circle directions, flatland HG g = 0.5,
eps = 0.01, lognormal sigma_T (Gaussian random field, std 0.5, correlation
length 0.1), sigma_a = 0.05, q = 1, unit inflow on the left edge; 4-level
MgNet with 32 channels and seeded weights; FGMRES(30) to a relative FP64
residual of 1e-6.  One step = one complete solve from x = 0 with inputs
already resident in HBM.  `value` is BF16-MgNet solves per second; the FP32
MgNet path is timed the same way beside it.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, GB/s
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, p):
    return float(np.percentile(np.asarray(xs), p)) if xs else None


def cpu_baseline(prob, blob, gpu_iters, budget_s):
    """The FP64 oracle on the host: a bounded run of FGMRES iterations, scaled to solves/s."""
    from oracle import solve as osolve
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    P = osolve.Problem(prob, blob)
    t0 = time.perf_counter()
    P.precond(P.b.reshape(-1))          # one V-cycle to size the sample
    P.apply(P.b.reshape(-1))
    per = time.perf_counter() - t0
    iters = int(max(3, min(60, budget_s / max(per, 1e-3))))
    t0 = time.perf_counter()
    _, st = P.solve(rtol=1e-30, restart=30, max_iters=iters)
    dt = time.perf_counter() - t0
    s_per_iter = dt / st["iterations"]
    return {
        "value": 1.0 / (s_per_iter * gpu_iters),
        "unit": "solves/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": "%d MgNet-preconditioned FGMRES(30) iterations of the same workload in FP64 NumPy "
                  "(%.1f s, %.3f s/iteration), scaled by the GPU's %.0f iterations per solve"
                  % (st["iterations"], dt, s_per_iter, gpu_iters),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--prof", default="conv", help="kernel class timed with events: conv|orth|apply|none")
    ap.add_argument("--prof-every", type=int, default=8, help="time every k-th launch of that class")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this solver has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_23265_amd import _lib as L
    from paper_2604_23265_amd import api
    from rte_inputs import configs, weights

    torch.cuda.set_device(0)
    prob = configs.c2(0)
    hdr, t = configs.problem_weights(prob)
    blob = weights.pack_mgn1(hdr, t)
    model = api.Model(blob)
    op = api.Operator(prob, model=model)
    kw = dict(restart=30, rtol=1e-6, max_iters=20000)
    ws = torch.empty(op.workspace_bytes(model, precond="bf16", **kw), dtype=torch.uint8, device="cuda")
    psi = torch.empty(op.n, dtype=torch.float64, device="cuda")

    def run(mode, steps, prof_cls=None):
        lat, its, res = [], [], []
        if prof_cls is not None:
            api.prof_reset()
            api.prof_enable(prof_cls, args.prof_every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            _, st = op.solve(model=model, psi=psi, workspace=ws, precond=mode, **kw)
            lat.append((time.perf_counter() - s0) * 1e3)
            its.append(st["iterations"])
            res.append(st["rel_residual"])
            if not st["converged"]:
                raise RuntimeError("solve did not converge: %r" % (st,))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = None
        if prof_cls is not None:
            api.prof_enable(prof_cls, 0)
            prof = api.prof_query(prof_cls)
        return dt, lat, its, res, prof

    log("warmup: %d BF16-path solves" % args.warmup)
    for _ in range(args.warmup):
        op.solve(model=model, psi=psi, workspace=ws, precond="bf16", **kw)
    classes = {"conv": L.K_CONV, "orth": L.K_ORTH, "apply": L.K_APPLY, "none": None}
    pc = classes[args.prof]
    log("timed: %d BF16-path solves (events on kernel class %s)" % (args.steps, args.prof))
    dt, lat, its, res, prof = run("bf16", args.steps, pc)
    value = args.steps / dt
    out = {
        "metric": "GMRES solves/s at 1e-6 rel residual, BF16 MgNet vs FP32; p50/p99 latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": "2D 128x128 grid, 32 directions, HG g=0.5, eps=0.01, lognormal GRF sigma_T "
                        "(std 0.5, corr 0.1), sigma_a=0.05, q=1, unit left inflow; 4-level MgNet, "
                        "32 channels, seeded weights; FGMRES(30), FP64 Arnoldi, rtol 1e-6",
            "grid": [128, 128], "directions": 32, "unknowns": int(op.n), "restart": 30, "rtol": 1e-6,
            "precond": "MgNet BF16 MFMA, FP32 accumulation",
        },
        "iterations_per_solve": float(np.mean(its)),
        "rel_residual_max": float(np.max(res)),
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
    }
    if prof is not None:
        ms, launches, work = prof
        avg_ms = ms / max(launches, 1)
        if args.prof == "conv":
            achieved = work / (ms * 1e-3) / 1e12
            out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": MFMA_PEAK_TFLOPS["bf16"],
                               "unit": "TFLOP/s", "frac": achieved / MFMA_PEAK_TFLOPS["bf16"],
                               "traffic": None, "kernel": "conv_kernel (implicit-GEMM 3x3/stride-2/"
                               "transposed convs of the V-cycle, BF16 MFMA)",
                               "timed_launches": launches, "sampling": "every %d-th launch" % args.prof_every,
                               "avg_launch_us": avg_ms * 1e3,
                               "work_per_launch": work / max(launches, 1), "work_unit": "FLOP"}
        else:
            achieved = work / (ms * 1e-3) / 1e9
            out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": args.prof,
                               "timed_launches": launches, "sampling": "every %d-th launch" % args.prof_every,
                               "avg_launch_us": avg_ms * 1e3,
                               "work_per_launch": work / max(launches, 1), "work_unit": "byte"}
    if not args.no_fp32:
        log("timed: %d FP32-path solves" % args.steps)
        dt32, lat32, its32, res32, _ = run("fp32", args.steps)
        out["fp32_path"] = {"value": args.steps / dt32, "unit": "solves/s", "ms_per_step": dt32 / args.steps * 1e3,
                            "iterations_per_solve": float(np.mean(its32)),
                            "latency_ms": {"p50": percentile(lat32, 50), "p99": percentile(lat32, 99)}}
        out["bf16_over_fp32"] = value / out["fp32_path"]["value"]
    if not args.no_cpu_baseline:
        log("cpu_baseline: oracle sample (~%.0f s)" % args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(prob, blob, float(np.mean(its)), args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
