#!/usr/bin/env python3
"""Benchmark: seconds to KKT tolerance 1e-8 of the interior-point solve of the
scenario absorber design NLP at 10 stages x 5000 scenarios, on one GPU.

One step = one complete cold-started IPM solve (evaluation, KKT assembly and
block LDL^T, Schur complement on d, solves, refinement, line search, until
E_0 <= 1e-8) with the feed table already resident on the device.

Prints one JSON line (see the fields below).  The CPU baseline times the
oracle on a bounded sample of the same workload and scales it to the metric.
"""

from __future__ import annotations

import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "s to 1e-8 KKT tol @5000 scenarios, cold vs NN warm start; FP64 MFMA util"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6


def factor_algorithmic(N: int, S: int) -> dict:
    """Algorithmic work of one launch of the block-LDL^T kernel (fused solve).

    Per stage: the 61-column frontal matrix (43 own unknowns, 16 coupling
    unknowns of the stage above, 2 right-hand sides) eliminated over 43 pivots:
    2 * sum_{m=18}^{60} m^2 flops; the backward sweep: 2 solves x 43 pivots x
    59-entry dot products.  Bytes: the stage record read (199 doubles) plus the
    43 stored pivot columns of 61 values written once and read back once by the
    backward sweep, plus right-hand side, diagonals and the two solutions
    (43 + 22 + 86 doubles).
    """
    flops_stage = 2 * sum(m * m for m in range(18, 61)) + 2 * 2 * 43 * 59
    bytes_stage = 8 * (199 + 2 * 43 * 61 + 43 + 22 + 86)
    return {"flops": flops_stage * N * S, "bytes": bytes_stage * N * S,
            "flops_per_stage": flops_stage, "bytes_per_stage": bytes_stage}


def kernel_source_hash() -> str:
    """Hash of the factor kernel's code (its source and the model header with
    comments and blank space removed): a change of comments keeps the counters."""
    h = hashlib.sha256()
    for f in ("factor.hip", "model.h"):
        with open(os.path.join(ROOT, "paper_2607_15420_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(N: int, S: int):
    """HBM bytes per factor launch from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_factor_C3_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("N") != N or t.get("S") != S:
        return None
    return t.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(params, feeds, N, iters_gpu, n_scen_sample):
    """The oracle IPM (as it stands) solved to E_0 <= 1e-8 from the cold start on
    the first n_scen_sample scenarios of the workload, timed on one thread and
    with every host core allowed (torch and BLAS thread pools); the whole-workload
    figure scales the measured seconds per scenario and iteration to all
    scenarios and to the iteration count of the GPU solve (an extrapolation,
    labelled as such)."""
    from threadpoolctl import threadpool_limits
    import torch
    from oracle import ipm as oipm

    S = feeds.shape[0]
    cores = os.cpu_count() or 1
    runs = {}
    for threads in (1, cores):
        torch.set_num_threads(threads)
        with threadpool_limits(limits=threads):
            prob = oipm.Problem(params, feeds[:n_scen_sample], N)
            t0 = time.perf_counter()
            r = oipm.OracleIPM(prob).solve()
            dt = time.perf_counter() - t0
        runs[threads] = {"seconds": dt, "iterations": r.iterations, "status": r.status, "E0": r.E0,
                         "per_scenario_iteration_s": dt / (n_scen_sample * max(r.iterations, 1))}
    best = min(runs, key=lambda t: runs[t]["seconds"])
    q = runs[best]
    est = q["per_scenario_iteration_s"] * S * iters_gpu
    return {
        "value": est, "unit": "s", "cores": best, "kind": "oracle",
        "sample": (f"oracle IPM from the cold start to E_0 <= 1e-8 on the first {n_scen_sample} of {S} scenarios: "
                   f"{q['iterations']} iterations in {q['seconds']:.1f} s with {best} thread(s); value = the "
                   f"measured seconds per scenario-iteration x {S} scenarios x the {iters_gpu} iterations of the "
                   f"GPU solve (extrapolated)"),
        "sample_seconds": q["seconds"],
        "one_thread": runs[1],
        "all_cores": runs[cores],
        "host_cores": cores,
        "host_cpu": cpu_model(),
    }


def measured_counters(N: int, S: int):
    """MFMA counter readings of the factor kernel from the committed rocprofv3
    summary, or None when the kernel source changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "k_factor_C3_mfma.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("N") != N or t.get("S") != S:
        return None
    return t


def warm_leg(params, steps: int, epochs: int):
    """Warm start at 10 stages x 5000 scenarios (seed 3): the network is trained
    on the converged states of the 20000 training scenarios (seed 4), then the
    warm-started solve (feature extraction + inference + IPM, cold fallback) is
    timed against the cold-started solve of the same instance."""
    import torch
    from absorber_inputs import CONFIGS, feed_table, perturbations
    from absorber_inputs.scenarios import TRAIN_SET
    from paper_2607_15420_amd import Absorber, Mlp

    dev = "cuda:0"
    N = TRAIN_SET.n_stages
    # training data: one single-scenario problem per training scenario, solved as one batch
    Ftr = TRAIN_SET.feeds(params)
    t0 = time.perf_counter()
    htr = Absorber.batch(params, [(N, Ftr[i:i + 1]) for i in range(Ftr.shape[0])])
    xtr = torch.empty(htr.nx, dtype=torch.float64, device=dev)
    ltr = torch.empty(htr.nc, dtype=torch.float64, device=dev)
    rc_tr, res_tr = htr.batch_solve(x_out=xtr, lam_out=ltr)
    Xtr = torch.empty((TRAIN_SET.n_scen, 3), dtype=torch.float32, device=dev)
    Ttr = torch.empty((TRAIN_SET.n_scen, 43 * N), dtype=torch.float32, device=dev)
    htr.warm_features(Xtr)
    htr.warm_targets(xtr, Ttr, ltr)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    n_ok = sum(r.status == 0 for r in res_tr)
    htr.close()
    print(f"bench: {n_ok} of {len(res_tr)} training problems solved in {t_data:.2f} s", file=sys.stderr, flush=True)
    net = Mlp(3, 256, 3, 43 * N, max_batch=512, seed=0)
    tr = net.train(Xtr, Ttr, net.default_train_options(epochs=epochs, batch=512, lr=1e-3))
    w = CONFIGS["C4"]
    h = Absorber(params, w.n_stages, w.feeds(params))
    opts = Absorber.default_options()
    h.ipm_solve(opts)  # warm-up of both paths
    h.warm_solve(net, opts)
    torch.cuda.synchronize()
    tc = time.perf_counter()
    for _ in range(steps):
        rc = h.ipm_solve(opts)
    torch.cuda.synchronize()
    cold_s = (time.perf_counter() - tc) / steps
    tw = time.perf_counter()
    for _ in range(steps):
        rw, used = h.warm_solve(net, opts)
    torch.cuda.synchronize()
    warm_s = (time.perf_counter() - tw) / steps
    h.close()
    net.close()
    return {
        "workload": f"{w.name}: {w.n_stages} stages x {w.n_scen} scenarios, feeds +-{int(w.amplitude * 100)}%, "
                    f"seed {w.seed}; network 3-256-256-256-{43 * N} (states and multipliers), bf16 MFMA, trained on "
                    f"{TRAIN_SET.n_scen} single-scenario solutions (seed {TRAIN_SET.seed}) from one batched solve",
        "cold_s": cold_s, "warm_s": warm_s, "speedup": cold_s / warm_s,
        "cold_iterations": rc.iterations, "warm_iterations": rw.iterations, "warm_used": used,
        "warm_feasibility_restarts": rw.feasibility_restarts,
        "cold_converged": rc.status == 0 and rc.E0 <= 1e-8, "warm_converged": rw.status == 0 and rw.E0 <= 1e-8,
        "warm_E0": rw.E0, "d_cold": rc.d, "d_warm": rw.d,
        "datagen_s": t_data, "datagen_converged": int(n_ok), "datagen_max_iterations": int(max(r.iterations for r in res_tr)),
        "train_s": tr.seconds, "train_steps": tr.steps,
        "train_epochs": epochs, "train_final_loss": tr.final_loss,
    }


def batch_leg(params, n_problems: int, sequential: bool):
    """64 independent design problems (stages uniform in 8-60, scenarios
    log-uniform in 50-2000, feeds +-15%, seed 5) solved as one batch, against
    solving them one after another with the same solver."""
    import numpy as np
    import torch
    from absorber_inputs import batch_problems, feed_table
    from paper_2607_15420_amd import Absorber

    probs = [(N, feed_table(pert, params)) for N, pert in batch_problems()[:n_problems]]
    n_chains = sum(f.shape[0] for _, f in probs)
    n_stages = sum(N * f.shape[0] for N, f in probs)
    opts = Absorber.default_options()
    h = Absorber.batch(params, probs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, res = h.batch_solve(opts)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    tuning = h.tuning()
    # the same batch with the per-problem decisions on the device and the
    # iterations replayed as captured graphs (same handle: tuned shapes kept)
    t0 = time.perf_counter()
    rc_g, res_g = h.batch_solve(Absorber.default_options(use_graph=1))
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    h.close()
    out = {
        "workload": f"C5: {len(probs)} problems, stages uniform 8-60, scenarios log-uniform 50-2000, feeds +-15%, "
                    f"seed 5 ({n_chains} scenarios, {n_stages} stages in all)",
        "batched_s": t_batch, "batched_converged": int(sum(r.status == 0 for r in res)),
        "batched_restarted": int(sum(r.feasibility_restarts for r in res)),
        "batched_solves_per_s": len(probs) / t_batch,
        "tuning": tuning,
        "graph_s": t_graph, "graph_converged": int(sum(r.status == 0 for r in res_g)),
        "graph_solves_per_s": len(probs) / t_graph,
        "graph_replays": int(max(r.graph_replays for r in res_g)),
        "graph_d_agree_1e-8": int(sum(a.status == 0 and b.status == 0 and abs(a.d - b.d) <= 1e-8 * a.d
                                      for a, b in zip(res, res_g))),
        "max_iterations": int(max(r.iterations for r in res)),
        "max_lin_resid": float(max(r.max_lin_resid for r in res)),
        "lin_resid_le_1e-10": int(sum(r.max_lin_resid <= 1e-10 for r in res)),
        "lin_resid_per_problem": [float(r.max_lin_resid) for r in res],
    }
    print(f"bench: batch of {len(probs)} solved in {t_batch:.2f} s", file=sys.stderr, flush=True)
    if sequential:
        t_seq, conv, d_agree = 0.0, 0, 0
        for p, (N, F) in enumerate(probs):
            hs = Absorber(params, N, F)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = hs.ipm_solve(opts)
            torch.cuda.synchronize()
            t_seq += time.perf_counter() - t0
            hs.close()
            conv += r.status == 0
            if r.status == 0 and res[p].status == 0 and abs(r.d - res[p].d) <= 1e-6 * r.d:
                d_agree += 1
            if p % 8 == 7:
                print(f"bench: sequential {p + 1}/{len(probs)}, {t_seq:.1f} s", file=sys.stderr, flush=True)
        out.update({"sequential_s": t_seq, "sequential_converged": int(conv),
                    "sequential_solves_per_s": len(probs) / t_seq, "speedup": t_seq / t_batch,
                    "d_agree_1e-6": int(d_agree)})
    return out


def extensions_leg(params, steps: int):
    """The model extensions at the benchmarked size (10 stages x 5000 scenarios,
    cold start, default options), each timed over `steps` solves after one
    warm-up: one diameter per column section (p = 4), the expected operating cost
    at a weight that puts the optimum 30% above the hydraulic bound, a specified
    pressure drop of 2000 Pa per stage, and scenarios drawn as convex
    combinations of seven base cases (C6)."""
    import copy
    import torch
    from absorber_inputs import CONFIGS
    from paper_2607_15420_amd import Absorber

    dev = "cuda:0"
    c3 = CONFIGS["C3"]
    F3 = c3.feeds(params)
    N = c3.n_stages

    def run(make, label):
        h = make()
        x = torch.empty(h.nx, dtype=torch.float64, device=dev)
        opts = Absorber.default_options()
        h.ipm_solve(opts, x_out=x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = [h.ipm_solve(opts, x_out=x) for _ in range(steps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        design = x[h.nx - h.npar:].cpu().tolist()
        h.close()
        r = rs[-1]
        print(f"bench: extension {label}: {1000 * dt:.1f} ms", file=sys.stderr, flush=True)
        return {"s": dt, "converged": all(q.status == 0 and q.E0 <= 1e-8 for q in rs), "iterations": r.iterations,
                "E0": r.E0, "max_lin_resid": r.max_lin_resid, "design": design}

    out = {"workload": "10 stages x 5000 scenarios (C3 feeds unless stated), cold start"}
    out["sections_p4"] = run(lambda: Absorber.sections(params, N, F3, 4), "4 sections")
    # operating cost: the weight at which the blower optimum sits 30% above the
    # hydraulic bound of the C3 solve (a single diameter)
    h = Absorber(params, N, F3)
    x = torch.empty(h.nx, dtype=torch.float64, device=dev)
    h.ipm_solve(Absorber.default_options(), x_out=x)
    d_hyd = float(x[-1])
    h.close()
    Mg = params["operating_cost"]["molar_mass"]
    K = params["operating_cost"]["loss_coef"]
    R = params["R"]
    p_in = F3[:, 17]
    Q = F3[:, 0] * R * F3[:, 5] / p_in
    rho = p_in * (F3[:, 1:5] @ Mg) / (R * F3[:, 5])
    a1 = 8.0 * K * N / math.pi ** 2 * float((rho * Q ** 3).mean())
    pop = copy.deepcopy(params)
    pop["operating_cost"]["weight"] = (1.3 * d_hyd) ** 5 / (4.0 * a1)
    out["operating_cost"] = run(lambda: Absorber(pop, N, F3), "operating cost")
    out["operating_cost"]["hydraulic_d"] = d_hyd
    out["operating_cost"]["blower_optimum"] = (4.0 * a1 * pop["operating_cost"]["weight"]) ** 0.2
    pdp = copy.deepcopy(params)
    pdp["dp_stage"] = 2000.0
    out["pressure_drop_2000Pa"] = run(lambda: Absorber(pdp, N, c3.feeds(pdp)), "pressure drop")
    c6 = CONFIGS["C6"]
    out["convex_scenarios_C6"] = run(lambda: Absorber(params, c6.n_stages, c6.feeds(params)), "C6")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-scen", type=int, default=16)
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-start leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-problems leg")
    ap.add_argument("--no-ext", action="store_true", help="skip the model-extensions leg")
    ap.add_argument("--batch-problems", type=int, default=64)
    ap.add_argument("--no-sequential", action="store_true", help="batched leg without the sequential comparison")
    ap.add_argument("--warm-epochs", type=int, default=300)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 8, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the scenario "
              "sharding over several GPUs is a design, not an implemented path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from absorber_inputs import CONFIGS, load_params
    from paper_2607_15420_amd import Absorber

    params = load_params()
    w = CONFIGS[args.config]
    feeds = w.feeds(params)
    N, S = w.n_stages, feeds.shape[0]
    torch.cuda.init()
    h = Absorber(params, N, feeds)
    x = torch.empty(h.nx, dtype=torch.float64, device="cuda:0")
    opts = Absorber.default_options()
    for _ in range(args.warmup):
        r = h.ipm_solve(opts, x_out=x)
    torch.cuda.synchronize()
    h.profile_enable(True, mask=1)  # time the factorisation kernel with events on its stream
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results.append(h.ipm_solve(opts, x_out=x))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = h.profile()
    h.profile_enable(False)
    r = results[-1]
    ok = all(q.status == 0 and q.E0 <= 1e-8 for q in results)
    ms_per_step = 1000.0 * elapsed / args.steps
    alg = factor_algorithmic(N, S)
    fac = prof["factor"]
    avg_ms = fac["ms"] / max(fac["calls"], 1)
    achieved = alg["bytes"] / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(N, S)
    mfma = measured_counters(N, S)
    out = {
        "metric": METRIC,
        "value": ms_per_step / 1000.0,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {N} stages x {S} scenarios, feeds +-{int(w.amplitude * 100)}% "
                               f"around nominal, seed {w.seed}, cold start", "n_stages": N, "n_scen": S,
                   "start": "cold"},
        "converged": ok,
        "iterations": r.iterations,
        "tuning": h.tuning(),
        "E0": r.E0,
        "d": r.d,
        "max_lin_resid": r.max_lin_resid,
        "roofline": {
            "kernel": "k_factor (block LDL^T + fused solve)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "avg_launch_ms": avg_ms,
            "launches": fac["calls"],
            "algorithmic_bytes": alg["bytes"],
            "fp64_tflops": alg["flops"] / (avg_ms * 1e-3) / 1e12,
            "fp64_frac": alg["flops"] / (avg_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            # FP64 MFMA utilisation from the committed counter reading of this kernel
            # (SQ_INSTS_VALU_MFMA_MOPS_F64, SQ_VALU_MFMA_BUSY_CYCLES); null when stale
            "mfma_frac": mfma["mfma_busy_frac"] if mfma else None,
            "mfma_counters": mfma,
        },
        "context": {"paper_h200_s": 33.3, "paper_ipopt_ma57_1thread_s": 695.5,
                    "paper_hardware": "1x H200 / Xeon 8568Y+ 1 thread; other model constants and data"},
    }
    h.close()
    print(f"bench: headline {ms_per_step:.1f} ms per solve", file=sys.stderr, flush=True)
    if not args.no_warm:
        out["warm_start"] = warm_leg(params, args.steps, args.warm_epochs)
        print("bench: warm-start leg done", file=sys.stderr, flush=True)
    if not args.no_batch:
        out["batch"] = batch_leg(params, args.batch_problems, not args.no_sequential)
    if not args.no_ext:
        out["extensions"] = extensions_leg(params, args.steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(params, feeds, N, r.iterations, args.cpu_scen)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
