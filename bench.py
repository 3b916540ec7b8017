"""Throughput of MgNet-preconditioned flexible GMRES on one MI355X.

Workload: 128x128 cells, 32 circle directions, flatland HG g = 0.5,
eps = 0.01, lognormal sigma_T (Gaussian random field, std 0.5, correlation
length 0.1), sigma_a = 0.05, q = 1, unit inflow on the left edge; 4-level
MgNet with 32 channels and seeded weights; FGMRES(30) to a relative FP64
residual of 1e-6.  One step = a batch of independent instances of this
family (media seeds 2000 + s) solved from x = 0 through the
continuous-batching server, inputs already resident in HBM.  `value` is
BF16-MgNet solves per second over the whole job; the FP32 MgNet path is
timed the same way beside it, and one instance solved alone is reported as
`single_solve`.  The MgNet weights are the ones trained offline for this
family (paper_2604_23265_amd/weights/c2_mgnet.mgn1, media seeds disjoint
from the benchmark's); the seeded initial weights are timed beside them.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import contextlib
import gc
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
CONV_SOURCE = os.path.join(ROOT, "paper_2604_23265_amd", "csrc", "mgnet.hip")
TRAINED = os.path.join(ROOT, "paper_2604_23265_amd", "weights", "c2_mgnet.mgn1")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "conv_tile_kernel_c2_traffic.md")


def measured_traffic():
    """(HBM bytes per conv launch, algorithmic bytes per launch of the same
    launches) from the committed counter summary, or (None, None).

    The summary records the SHA-256 of the convolution source it was taken
    with; a changed kernel makes the figures stale, so they are not reported.
    """
    import hashlib
    try:
        src = hashlib.sha256(open(CONV_SOURCE, "rb").read()).hexdigest()
        fields = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip()
        if fields.get("source-sha256") != src:
            return None, None
        return float(fields["hbm-bytes-per-launch"]), float(fields["algorithmic-bytes-per-launch"])
    except (OSError, KeyError, ValueError):
        return None, None


APPLY_SOURCE = os.path.join(ROOT, "paper_2604_23265_amd", "csrc", "apply.hip")
APPLY_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_mfma_kernel_c4_c5.md")


def measured_apply_traffic():
    """{case name: HBM bytes per FP32 apply launch} from the committed counter
    summary of the large cases, or {} when the apply source has changed since."""
    import hashlib
    try:
        src = hashlib.sha256(open(APPLY_SOURCE, "rb").read()).hexdigest()
        fields = {}
        for line in open(APPLY_TRAFFIC_FILE):
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip()
        if fields.get("source-sha256") != src:
            return {}
        pre = "hbm-bytes-per-launch-"
        return {k[len(pre):]: float(v) for k, v in fields.items() if k.startswith(pre)}
    except (OSError, ValueError):
        return {}


def trained_description():
    """How the C2 weights were trained, from their record next to the blob."""
    try:
        rec = json.load(open(TRAINED[:-len(".mgn1")] + ".json"))["record"]
        return ("trained offline for the C2 family (residual loss ||b - L M b||, AdamW, %d steps at lr %g "
                "over %d seeded media disjoint from these instances; weights/c2_mgnet.json)"
                % (rec["steps"], rec["lr"], rec["media"]))
    except (OSError, KeyError, ValueError):
        return "trained offline for the C2 family (weights/c2_mgnet.json)"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, p):
    return float(np.percentile(np.asarray(xs), p)) if xs else None


def host_cpu():
    """(logical CPUs, model name) of the host."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_baseline(prob, blob, gpu_iters, budget_s):
    """The FP64 oracle on the host: a bounded run of FGMRES iterations, scaled to solves/s."""
    from oracle import solve as osolve
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    ncpu, model = host_cpu()
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
        "host_cpus": ncpu, "cpu_model": model, "blas_threads": int(threads),
        "threads_note": "the convolutions' tensor contractions run on the BLAS threads; the stencil, the "
                        "elementwise network arithmetic and the Krylov loop run single-threaded in NumPy",
    }


def oracle_c1(api, torch, configs, weights):
    """The small workload as a full solve: the oracle (FP64 GMRES(20) with the FP64 V-cycle of a
    2-level seeded MgNet, rtol 1e-8) timed on the host, and the GPU's BF16 path beside it."""
    from oracle import solve as osolve
    prob = configs.c1()
    hdr, t = configs.problem_weights(prob)
    blob = weights.pack_mgn1(hdr, t)
    P = osolve.Problem(prob, blob)
    t0 = time.perf_counter()
    x, st = P.solve(rtol=1e-8, restart=20, max_iters=5000)
    dt = time.perf_counter() - t0
    model = api.Model(blob)
    op = api.Operator(prob, model=model)
    op.solve(model=model, precond="bf16", rtol=1e-8, restart=20)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    xg, sg = op.solve(model=model, precond="bf16", rtol=1e-8, restart=20)
    torch.cuda.synchronize()
    dg = time.perf_counter() - t1
    err = float(np.linalg.norm(xg.cpu().numpy() - x.reshape(-1)) / np.linalg.norm(x))
    return {"workload": "2D 32x32, 16 directions, g=0, eps=1, sigma_T 1 with a 10 inclusion, sigma_a 0.1, q=1 on "
                        "the inclusion; 2-level seeded MgNet (16 channels); GMRES(20) to 1e-8",
            "oracle_s": dt, "oracle_iterations": int(st["iterations"]), "oracle_converged": bool(st["converged"]),
            "gpu_bf16_ms": dg * 1e3, "gpu_iterations": int(sg["iterations"]),
            "gpu_vs_oracle_rel_error": err}


def solution_errors(prob, blob, xs):
    """Relative error of GPU solutions of one instance against the oracle's psi* (FP64 FGMRES with
    the FP64 V-cycle of the same weights, rtol 1e-12); xs: {label: host array}."""
    from oracle import solve as osolve
    P = osolve.Problem(prob, blob)
    t0 = time.perf_counter()
    ref, st = P.solve(rtol=1e-12, restart=30, max_iters=400)
    ref = ref.reshape(-1)
    out = {"reference": "oracle psi* of GRF seed 2000, FP64 FGMRES(30) + FP64 V-cycle to rtol 1e-12 "
                        "(%d iterations, %.1f s)" % (st["iterations"], time.perf_counter() - t0)}
    for k, x in xs.items():
        out[k] = {"rel_l2": float(np.linalg.norm(x - ref) / np.linalg.norm(ref)),
                  "rel_max": float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))}
    return out


@contextlib.contextmanager
def no_gc():
    """No garbage-collection pass inside a timed region: a full pass over this process's
    heap stalls the thread that submits and collects the solves."""
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()


def serving_leg(args, api, torch, configs, weights):
    """Served latency on the C3 stream: a closed batch measures saturated throughput, then
    Poisson arrivals at 0.7x that rate give arrival-to-completion p50/p99."""
    reqs = [configs.c3_request(r) for r in range(args.serving_requests)]
    models = {}
    used = {}
    ops = []
    builds = []
    for p in reqs:
        N = p["dirs"].shape[0]
        if N not in models:
            path = os.path.join(ROOT, "paper_2604_23265_amd", "weights", "c3_n%d.mgn1" % N)
            if args.weights == "trained" and os.path.exists(path):
                models[N] = api.Model(open(path, "rb").read())
                used[N] = "trained (weights/c3_n%d.mgn1)" % N
            else:
                hdr, t = configs.problem_weights(p)
                models[N] = api.Model(weights.pack_mgn1(hdr, t))
                used[N] = "seeded"
        tb = time.perf_counter()
        ops.append(api.Operator(p, model=models[N]))
        builds.append((time.perf_counter() - tb) * 1e3)
    outs = [torch.empty(op.n, dtype=torch.float64, device="cuda") for op in ops]
    kw = dict(restart=30, rtol=1e-6, max_iters=args.serving_max_iters, precond="bf16")
    srv = api.Server(arena_bytes=args.serving_arena_gb << 30, max_slots=args.serving_slots)

    def run(arrivals):
        t0 = time.perf_counter()
        pending = {}
        submitted = 0
        done = {}
        while len(done) < len(ops):
            now = time.perf_counter() - t0
            while submitted < len(ops) and arrivals[submitted] <= now:
                tk = srv.submit(ops[submitted], outs[submitted], model=ops[submitted].model, **kw)
                pending[tk] = (submitted, t0 + arrivals[submitted])
                submitted += 1
            for tk in list(pending):
                r = srv.poll(tk)
                if r is not None:
                    i, t_arr = pending.pop(tk)
                    done[i] = (time.perf_counter() - t_arr, r[0], r[1])
            time.sleep(0.0005)
        return time.perf_counter() - t0, done

    log("serving: closed batch of %d requests" % len(ops))
    with no_gc():
        wall, done = run([0.0] * len(ops))
    sat = len(ops) / wall
    rate = 0.7 * sat
    arr = list(configs.c3_arrivals(len(ops), rate=rate, seed=3999))
    arr = [a - arr[0] for a in arr]
    log("serving: Poisson arrivals at %.2f req/s" % rate)
    with no_gc():
        wall2, done2 = run(arr)
    lat = [d[0] * 1e3 for d in done2.values()]
    lat_b = [d[0] * 1e3 + builds[i] for i, d in done2.items()]
    its = [d[2]["iterations"] for d in done2.values()]
    ok = sum(1 for d in done2.values() if d[1] == 0)
    q = srv.query()
    srv.close()
    return {"requests": len(ops), "slots": args.serving_slots, "saturated_solves_per_s": sat,
            "arrival_rate": rate, "completed_ok": ok, "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
            "latency_note": "p50/p99: arrival to completion of the solve, operators built beforehand; "
                            "with_build: plus that request's operator build (host FP64 setup, upload, CoeffNet)",
            "build_ms": {"p50": percentile(builds, 50), "p99": percentile(builds, 99)},
            "with_build_ms": {"p50": percentile(lat_b, 50), "p99": percentile(lat_b, 99)},
            "iterations_mean": float(np.mean(its)), "iterations_max": int(np.max(its)),
            "arena_peak_gb": q["arena_peak"] / 2 ** 30, "max_iters": args.serving_max_iters,
            "weights": {str(k): v for k, v in sorted(used.items())},
            "stream": "seeded C3 draws: grid {64,128,256}^2, 16/32 directions, eps log-uniform [1e-3,1], "
                      "g ~ U[0,0.8], lognormal GRF sigma_T; BF16 MgNet FGMRES(30) to 1e-6"}


def large_leg(args, api, L, torch, configs, weights):
    """Kernel rates of the large single solves (the 512^2 x 64-direction and the 64^3 x
    96-direction cases) with seeded weights: the FP32 operator apply, the BF16 V-cycle and
    its convolutions, and the time per FGMRES iteration of a bounded solve."""
    def ev_time(fn, reps):
        for _ in range(3):
            fn()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps * 1e-3

    out = {}
    cases = (("512x512_64dir", configs.c4, 30,
              "2D 512x512, 64 directions, HG g=0.9, eps=1e-3, 8x8 checkerboard sigma_T {1,100}; "
              "5-level MgNet, 64 channels"),
             ("64x64x64_96dir", configs.c5, 20,
              "3D 64^3, 96 sphere directions, HG g=0.8, eps=1e-2, lognormal GRF sigma_T; "
              "4-level 3D MgNet, 48 channels"))
    for name, make, k, desc in cases:
        log("large: %s" % name)
        prob = make()
        hdr, t = configs.problem_weights(prob)
        model = api.Model(weights.pack_mgn1(hdr, t))
        op = api.Operator(prob, model=model)
        torch.cuda.synchronize()
        x = torch.randn(op.n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        dt_apply = ev_time(lambda: op.apply(x, y), 20)
        apply_gbs = (8 * op.n + 8 * op.cells) / dt_apply / 1e9
        x64 = torch.randn(op.n, dtype=torch.float64, device="cuda")
        r64 = torch.empty_like(x64)
        dt_res = ev_time(lambda: op.residual(x64, r64), 20)
        res_gbs = (24 * op.n + 16 * op.cells) / dt_res / 1e9
        del x64, r64
        v = torch.randn(op.n, dtype=torch.float64, device="cuda")
        ws = torch.empty(op.precond_workspace(model), dtype=torch.uint8, device="cuda")
        z = op.precond(model, v, mode="bf16", workspace=ws)
        dt_mg = ev_time(lambda: op.precond(model, v, mode="bf16", z=z, workspace=ws), 5)
        api.prof_reset()
        api.prof_enable(L.K_CONV, 1)
        for _ in range(3):
            op.precond(model, v, mode="bf16", z=z, workspace=ws)
        torch.cuda.synchronize()
        api.prof_enable(L.K_CONV, 0)
        ms, n, work, nb = api.prof_query(L.K_CONV)
        ckeys = api.prof_query_keys(L.K_CONV)
        api.prof_reset()
        # per V-cycle level (the key is floor(log2(output channels)); the channel counts
        # are c0 times a power of two): achieved rates and where the intensity sits
        # against the ridge
        c0 = int(prob["mgnet"]["c0"])
        lg0 = c0.bit_length() - 1
        ridge = MFMA_PEAK_TFLOPS["bf16"] * 1e12 / (HBM_PEAK_GBS * 1e9)
        by_level = {}
        for key, (kms, kn, kwork, kb) in sorted(ckeys.items()):
            t_k, g_k = kwork / (kms * 1e-3) / 1e12, kb / (kms * 1e-3) / 1e9
            by_level["cout_%d" % (c0 << max(0, key - lg0))] = {
                "launches": kn, "avg_us": kms / kn * 1e3, "share_of_conv_time": kms / ms,
                "TFLOPs": t_k, "mfma_frac": t_k / MFMA_PEAK_TFLOPS["bf16"], "GBs_algorithmic": g_k,
                "hbm_frac": g_k / HBM_PEAK_GBS, "intensity_flop_per_byte": kwork / kb,
                "bound": "mfma" if kwork / kb >= ridge else "hbm"}
        xs, st = op.solve(model=model, precond="bf16", rtol=1e-12, restart=k, max_iters=40)
        out[name] = {
            "workload": desc, "unknowns": int(op.n), "weights": "seeded (seed of the workload)",
            "apply_fp32_us": dt_apply * 1e6, "apply_fp32_GBs": apply_gbs, "apply_frac_hbm": apply_gbs / HBM_PEAK_GBS,
            "apply_bytes": "4 B in + 4 B out per unknown + 8 B per cell",
            "residual_fp64_us": dt_res * 1e6, "residual_fp64_GBs": res_gbs,
            "residual_fp64_frac_hbm": res_gbs / HBM_PEAK_GBS,
            "residual_bytes": "8 B x + 8 B b in + 8 B r out per unknown + 16 B per cell",
            "vcycle_bf16_ms": dt_mg * 1e3,
            "conv_launches_per_vcycle": n / 3, "conv_TFLOPs": work / (ms * 1e-3) / 1e12,
            "conv_mfma_frac": work / (ms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["bf16"],
            "conv_GBs": nb / (ms * 1e-3) / 1e9, "conv_frac_hbm": nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "conv_by_output_channels": by_level,
            "fgmres_restart": k, "fgmres_ms_per_iteration": st["ms_total"] / max(st["iterations"], 1),
            "rel_residual_after_40": st["rel_residual"],
        }
        hbm = measured_apply_traffic().get(name)
        if hbm is not None:
            # the same launch's HBM bytes from the committed counter summary
            alg = 8.0 * op.n + 8.0 * op.cells
            out[name]["apply_hbm_bytes_counters"] = hbm
            out[name]["apply_hbm_GBs_counters"] = hbm / dt_apply / 1e9
            out[name]["apply_traffic_over_algorithmic"] = hbm / alg
        del op, model, x, y, v, ws, z, xs
        torch.cuda.empty_cache()
    return out


def discretisation_leg(args, api, torch, configs):
    """The paper's own discretisations on the C2 medium (32 directions, eps = 0.01, the first
    GRF draw): the TFPS operator of Sec. 2.2 on 128^2 cells (build, y = A x, r = b - A x and
    the cell-centre values, FP64) and the adaptive scheme's maps of Sec. 2.3 / 3.4 at
    delta = 1e-2 on 64^2 cells (host build, compressed residual, layer reconstruction,
    filtered loss; at 128^2 nearly every function is kept and the host build takes a minute)."""
    def ev_time(fn, reps=20):
        for _ in range(3):
            fn()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps * 1e-3

    log("discretisations: TFPS operator build, 128^2 cells x 32 directions")
    prob = dict(configs.c2(0), scheme="tfps")
    torch.cuda.synchronize()
    tb = time.perf_counter()
    op = api.Operator(prob)
    torch.cuda.synchronize()
    build_tfps = time.perf_counter() - tb
    n, cells, N = op.n, op.cells, op.ndir
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    r = torch.empty_like(x)
    psi = torch.empty(N * cells, dtype=torch.float64, device="cuda")
    t_apply = ev_time(lambda: op.apply(x, y))
    t_res = ev_time(lambda: op.residual(x, r))
    t_cv = ev_time(lambda: op.cell_values(x, psi))
    # per unknown 8 B in and 8 B out (the residual also reads b); per cell its table id and sT;
    # every distinct eigen-basis table (2N x N eigenvector entries and 2N eigenvalues, FP64)
    # once -- on this medium every cell has its own ratio, so the tables dominate
    tables = op.info["nbasis"] * 2 * N * (N + 1) * 8.0
    b_apply = 16.0 * n + 12.0 * cells + tables
    b_res = 24.0 * n + 12.0 * cells + tables
    b_cv = 8.0 * n + 8.0 * N * cells + 12.0 * cells + tables
    out = {"workload": "128x128 cells, 32 directions, eps=0.01, C2 medium (GRF seed 2000); TFPS unknowns "
                       "2N per cell", "unknowns": int(n),
           "tfps": {"build_ms": build_tfps * 1e3,
                    "apply_us": t_apply * 1e6, "apply_GBs": b_apply / t_apply / 1e9,
                    "apply_frac_hbm": b_apply / t_apply / 1e9 / HBM_PEAK_GBS,
                    "residual_us": t_res * 1e6, "residual_GBs": b_res / t_res / 1e9,
                    "cell_values_us": t_cv * 1e6, "cell_values_GBs": b_cv / t_cv / 1e9,
                    "bases": int(op.info["nbasis"]), "basis_table_MB": tables / 1e6,
                    "bytes": "the basis tables once, plus: apply 16 B per unknown + 12 B per cell; residual "
                             "24 + 12; cell values 8 B per coefficient in, 8 B per value out"}}
    op.close()
    delta = 1e-2
    log("discretisations: ATFPS build, 64^2 cells x 32 directions, delta %g" % delta)
    prob = dict(configs.c2(0, n=64), scheme="tfps")
    op = api.Operator(prob)
    n, cells = op.n, op.cells
    tb = time.perf_counter()
    at = api.Atfps(op, delta)
    build_at = time.perf_counter() - tb
    log("discretisations: ATFPS maps timed")
    psi = torch.randn(N * cells, dtype=torch.float64, device="cuda")
    al = torch.randn(at.n_kept, dtype=torch.float64, device="cuda")
    rr = torch.empty(at.n_rows, dtype=torch.float64, device="cuda")
    coef = torch.empty(n, dtype=torch.float64, device="cuda")
    rho = torch.empty(at.n_rows, dtype=torch.float64, device="cuda")
    t_ar = ev_time(lambda: at.residual(al, rr))
    t_rc = ev_time(lambda: at.reconstruct(al, coef))
    t_fl = ev_time(lambda: at.filtered_loss(psi, rho))
    # sparse rows: per stored entry its value, column and the gathered operand; per row its two
    # offsets, the constant and the result.  The reconstruction and loss maps' entry counts are
    # not exported; their rates are reported as time only.
    b_ar = 20.0 * at.nnz + 32.0 * at.n_rows
    out["atfps"] = {"workload": "64x64 cells, 32 directions, eps=0.01, C2 medium family (GRF seed 2000)",
                    "delta": delta, "kept_unknowns": at.n_kept, "kept_fraction": at.n_kept / n,
                    "compressed_nnz": at.nnz, "build_ms": build_at * 1e3,
                    "residual_us": t_ar * 1e6, "residual_GBs": b_ar / t_ar / 1e9,
                    "residual_frac_hbm": b_ar / t_ar / 1e9 / HBM_PEAK_GBS,
                    "reconstruct_us": t_rc * 1e6, "filtered_loss_us": t_fl * 1e6,
                    "bytes": "compressed residual: 20 B per stored entry + 32 B per row"}
    at.close()
    op.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed batches")
    ap.add_argument("--warmup", type=int, default=2, help="untimed batches")
    ap.add_argument("--weights", default="trained", choices=["trained", "seeded"],
                    help="MgNet weights: trained offline for the family, or the seeded initial ones")
    ap.add_argument("--batch", type=int, default=32, help="independent instances per step")
    ap.add_argument("--arena-gb", type=float, default=16.0)
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-comparators", action="store_true",
                    help="skip the Block-Jacobi and unpreconditioned batches")
    ap.add_argument("--prof", default="conv", help="kernel class timed with events: conv|orth|apply|none")
    ap.add_argument("--prof-every", type=int, default=1,
                    help="in the timed batch, run every k-th Arnoldi step without its graph and time it")
    ap.add_argument("--prof-batch", type=int, default=-1,
                    help="the timed batch whose steps are timed (default: the middle one)")
    ap.add_argument("--no-large", action="store_true", help="skip the large single-solve kernel rates")
    ap.add_argument("--no-tfps", action="store_true", help="skip the TFPS / ATFPS rates")
    ap.add_argument("--serving-requests", type=int, default=512, help="requests of the C3 stream (0 = skip)")
    ap.add_argument("--serving-slots", type=int, default=16)
    ap.add_argument("--serving-arena-gb", type=int, default=32)
    ap.add_argument("--serving-max-iters", type=int, default=3000)
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="bytes of a plain device copy run before the solves (reference for counter scaling)")
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
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # the C2 family: media seeds 2000 + s, s = 0 .. batch-1, one seeded network
    probs = [configs.c2(s) for s in range(args.batch)]
    hdr, t = configs.problem_weights(probs[0])
    seeded_blob = weights.pack_mgn1(hdr, t)
    blob = open(TRAINED, "rb").read() if args.weights == "trained" else seeded_blob
    model = api.Model(blob)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    ops = [api.Operator(p, model=model) for p in probs]
    build_ms = (time.perf_counter() - tb) * 1e3 / len(probs)
    kw = dict(restart=30, rtol=1e-6, max_iters=20000)
    outs = [torch.empty(op.n, dtype=torch.float64, device="cuda") for op in ops]
    srv = api.Server(arena_bytes=int(args.arena_gb * 2 ** 30), max_slots=args.batch)
    classes = {"conv": L.K_CONV, "orth": L.K_ORTH, "apply": L.K_APPLY, "none": None}
    pc = classes[args.prof]

    def batch(mode):
        """One step: every instance of the batch submitted at once and solved to rtol."""
        mdl = model if mode in ("bf16", "fp32") else None
        tk = [srv.submit(op, o, model=mdl, precond=mode, **kw) for op, o in zip(ops, outs)]
        res = {}
        while len(res) < len(tk):
            for x in tk:
                if x not in res:
                    r = srv.poll(x)
                    if r is not None:
                        res[x] = r
            time.sleep(0.0002)
        sts = [res[x][1] for x in tk]
        if not all(s["converged"] for s in sts):
            raise RuntimeError("a solve did not converge: %r" % (sts,))
        return sts

    step_ms = []

    # the kernel-class timer runs during one timed batch (every prof_every-th tick
    # of it without its graph, its launches of the class timed): a whole batch
    # covers every phase of the solves once, and the other batches run as they
    # would untimed
    prof_batch = min(max(args.prof_batch if args.prof_batch >= 0 else args.steps // 2, 0), args.steps - 1)

    def run(mode, steps, prof_cls=None):
        if prof_cls is not None:
            api.prof_reset()
        with no_gc():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = []
            step_ms.clear()
            for i in range(steps):
                if prof_cls is not None and i == prof_batch:
                    api.prof_enable(prof_cls, args.prof_every)
                ts = time.perf_counter()
                sts += batch(mode)
                step_ms.append((time.perf_counter() - ts) * 1e3)
                if prof_cls is not None and i == prof_batch:
                    api.prof_enable(prof_cls, 0)
            torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = None
        if prof_cls is not None:
            prof = api.prof_query(prof_cls)
        return dt, sts, prof

    log("warmup: %d batches of %d BF16-path solves" % (args.warmup, args.batch))
    for _ in range(args.warmup):
        batch("bf16")
    log("timed: %d batches of %d BF16-path solves (events on kernel class %s)" % (args.steps, args.batch, args.prof))
    dt, sts, prof = run("bf16", args.steps, pc)
    bf16_step_ms = list(step_ms)
    log("step ms: " + " ".join("%.2f" % t for t in bf16_step_ms))
    conv_keys = api.prof_query_keys(L.K_CONV) if args.prof == "conv" else {}
    orth_keys = api.prof_query_keys(L.K_ORTH) if args.prof == "orth" else {}
    x_bf16 = outs[0].cpu().numpy()
    nsolves = args.steps * args.batch
    value = nsolves / dt
    lat = [s["ms_total"] for s in sts]
    its = [s["iterations"] for s in sts]
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
                        "32 channels; FGMRES(30), FP64 Arnoldi, rtol 1e-6",
            "step": "%d independent instances (GRF seeds 2000..%d) solved concurrently through the "
                    "continuous-batching server" % (args.batch, 2000 + args.batch - 1),
            "grid": [128, 128], "directions": 32, "unknowns": int(ops[0].n), "restart": 30, "rtol": 1e-6,
            "precond": "MgNet BF16 MFMA, FP32 accumulation",
            "weights": trained_description() if args.weights == "trained" else "seeded initial weights (seed 2001)",
        },
        "iterations_per_solve": float(np.mean(its)),
        "rel_residual_max": float(max(s["rel_residual"] for s in sts)),
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                       "note": "submission to completion inside a batch"},
        "step_ms": {"median": percentile(bf16_step_ms, 50), "p99": percentile(bf16_step_ms, 99),
                    "min": min(bf16_step_ms), "max": max(bf16_step_ms)},
        "operator_build_ms_per_solve": build_ms,
        "operator_build_note": "host FP64 setup, upload and CoeffNet per instance, outside the timed region",
    }
    if prof is not None:
        ms, launches, work, nbytes = prof
        avg_ms = ms / max(launches, 1)
        samp = ("timed batch %d of %d: %s run without its graph, every launch of the class in it timed"
                % (prof_batch + 1, args.steps,
                   "every Arnoldi step" if args.prof_every == 1 else "one Arnoldi step in %d" % args.prof_every))
        if args.prof == "conv":
            # The convolutions are bound by the matrix cores where their channel count
            # is 64 or more (3 of the 4 levels here): the headline is MFMA use against
            # the dense BF16 peak.  Per output-channel count (one V-cycle level each for
            # the smoothers) the achieved rates and the algorithmic intensity against the
            # ridge 2500 / 8 = 312 flop/B say which bound each level meets.
            gbs = nbytes / (ms * 1e-3) / 1e9
            tflops = work / (ms * 1e-3) / 1e12
            traffic, traffic_alg = measured_traffic()
            ridge = MFMA_PEAK_TFLOPS["bf16"] * 1e12 / (HBM_PEAK_GBS * 1e9)
            levels = {}
            for key, (kms, kn, kwork, kb) in sorted(conv_keys.items()):
                t_k, g_k = kwork / (kms * 1e-3) / 1e12, kb / (kms * 1e-3) / 1e9
                levels["cout_%d" % (1 << key)] = {
                    "launches": kn, "avg_us": kms / kn * 1e3, "share_of_conv_time": kms / ms,
                    "TFLOPs": t_k, "mfma_frac": t_k / MFMA_PEAK_TFLOPS["bf16"],
                    "GBs_algorithmic": g_k, "hbm_frac": g_k / HBM_PEAK_GBS,
                    "intensity_flop_per_byte": kwork / kb,
                    "bound": "mfma" if kwork / kb >= ridge else "hbm"}
            out["roofline"] = {"bound": "mfma", "achieved": tflops, "peak": MFMA_PEAK_TFLOPS["bf16"],
                               "unit": "TFLOP/s", "frac": tflops / MFMA_PEAK_TFLOPS["bf16"],
                               "traffic": traffic,
                               "traffic_unit": "HBM bytes per launch (counters, every launch of one batch)",
                               "traffic_over_algorithmic": (traffic / traffic_alg) if traffic else None,
                               "kernel": "conv_tile_kernel (3x3 stride-1/stride-2 and transposed 4x4 "
                                         "convolutions of the V-cycle, BF16 MFMA, all solves of the batch per launch)",
                               "timed_launches": launches, "sampling": samp,
                               "avg_launch_us": avg_ms * 1e3,
                               "flop_per_launch": work / max(launches, 1),
                               "algorithmic_bytes_per_launch": nbytes / max(launches, 1),
                               "intensity_flop_per_byte": work / max(nbytes, 1.0),
                               "hbm": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": gbs / HBM_PEAK_GBS,
                                       "bytes": "input, BF16 weights, output and FP32 epilogue tensors once"},
                               "by_output_channels": levels}
        else:
            achieved = work / (ms * 1e-3) / 1e9
            out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": args.prof,
                               "timed_launches": launches, "sampling": samp,
                               "avg_launch_us": avg_ms * 1e3,
                               "work_per_launch": work / max(launches, 1), "work_unit": "byte"}
            if orth_keys:
                names = {1: "dots", 2: "reduce", 3: "finish_dots (CGS2 pass 1)", 4: "updots (CGS2 pass 2)",
                         5: "finish (Givens)"}
                out["roofline"]["by_kernel"] = {
                    names.get(k, str(k)): {"launches": kn, "avg_us": kms / kn * 1e3,
                                           "algorithmic_bytes_per_launch": kb / kn,
                                           "GBs_algorithmic": kb / (kms * 1e-3) / 1e9,
                                           "hbm_frac": kb / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS}
                    for k, (kms, kn, kwork, kb) in sorted(orth_keys.items())}
    if not args.no_fp32:
        log("timed: %d batches of FP32-path solves" % args.steps)
        dt32, sts32, _ = run("fp32", args.steps)
        x_fp32 = outs[0].cpu().numpy()
        out["fp32_path"] = {"value": nsolves / dt32, "unit": "solves/s", "ms_per_step": dt32 / args.steps * 1e3,
                            "iterations_per_solve": float(np.mean([s["iterations"] for s in sts32])),
                            "latency_ms": {"p50": percentile([s["ms_total"] for s in sts32], 50),
                                           "p99": percentile([s["ms_total"] for s in sts32], 99)}}
        out["bf16_over_fp32"] = value / out["fp32_path"]["value"]
    if args.weights == "trained" and not args.no_comparators:
        # the seeded initial weights of the same network, one timed batch
        log("timed: 1 batch with the seeded weights")
        seeded = api.Model(seeded_blob)
        ops_s = [api.Operator(p, model=seeded) for p in probs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tk = [srv.submit(op, o, model=seeded, precond="bf16", **kw) for op, o in zip(ops_s, outs)]
        res = {}
        while len(res) < len(tk):
            for x in tk:
                if x not in res:
                    r = srv.poll(x)
                    if r is not None:
                        res[x] = r
            time.sleep(0.0002)
        dts = time.perf_counter() - t0
        out["seeded_weights"] = {"value": args.batch / dts, "unit": "solves/s",
                                 "iterations_per_solve": float(np.mean([res[x][1]["iterations"] for x in tk]))}
        del ops_s
    if not args.no_comparators:
        # the paper's comparators on the same batch: cell-wise Block-Jacobi
        # and no preconditioner (one timed batch each)
        comp = {}
        for mode, label in (("bj", "block_jacobi"), ("none", "unpreconditioned")):
            log("timed: 1 batch of %s solves" % label)
            dtc, stc, _ = run(mode, 1)
            comp[label] = {"value": args.batch / dtc, "unit": "solves/s",
                           "iterations_per_solve": float(np.mean([s["iterations"] for s in stc])),
                           "ms_per_step": dtc * 1e3}
        comp["mgnet_bf16_iterations_per_solve"] = float(np.mean(its))
        comp["note"] = ("FGMRES(30) to the same 1e-6 FP64 residual on the same batch; MgNet with the weights "
                        "of this run (%s) against the classical cell-wise Block-Jacobi and no preconditioner"
                        % args.weights)
        out["comparators"] = comp
    if not args.no_single:
        log("single solves: instance 0 alone, %d times" % args.steps)
        ws = torch.empty(ops[0].workspace_bytes(model, precond="bf16", **kw), dtype=torch.uint8, device="cuda")
        with no_gc():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, st = ops[0].solve(model=model, psi=outs[0], workspace=ws, precond="bf16", **kw)
            torch.cuda.synchronize()
        d1 = (time.perf_counter() - t0) / args.steps
        out["single_solve"] = {"value": 1.0 / d1, "unit": "solves/s", "ms": d1 * 1e3,
                               "iterations": st["iterations"], "instance": "GRF seed 2000"}
    srv.close()
    prob, blob = probs[0], blob
    if args.serving_requests:
        out["serving"] = serving_leg(args, api, torch, configs, weights)
    if not args.no_large:
        out["large_single_solves"] = large_leg(args, api, L, torch, configs, weights)
    if not args.no_tfps:
        out["discretisations"] = discretisation_leg(args, api, torch, configs)
    if not args.no_cpu_baseline:
        log("cpu_baseline: oracle sample (~%.0f s)" % args.cpu_budget)
        out["cpu_baseline"] = cpu_baseline(prob, blob, float(np.mean(its)), args.cpu_budget)
        log("oracle: psi* of instance 0 for the solution error")
        xs = {"bf16_path": x_bf16}
        if not args.no_fp32:
            xs["fp32_path"] = x_fp32
        out["solution_error_vs_oracle"] = solution_errors(prob, blob, xs)
        out["solution_error_vs_oracle"]["note"] = ("instance 0's solutions of the timed runs (rtol 1e-6) "
                                                   "against the oracle's psi*")
        log("oracle: the small workload as a full solve")
        out["c1_full_solve"] = oracle_c1(api, torch, configs, weights)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
