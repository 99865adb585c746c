"""Benchmark of the PinT-QBVM all-at-once solve on one MI355X.

Workload: 2D, Omega=(0,1)^2, m=255 interior points per dimension (5-point
Laplacian), n=256 backward-Euler steps (N_t = 257), T=1, alpha=1e-4, PinT-QBVM,
FP64; initial datum = 64 random lowest sine modes, 0.5% relative Gaussian noise
(seeded, synthetic).  One step = one full solve (every level, n+1 = 257 levels of
255^2 values), inputs resident in HBM.  Metric: solve throughput in Munknowns/s
on the n*m^d basis.

Prints one JSON line.  --gpus above 1 is refused: this build measures one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2107_06381_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str, variant: int):
    """HBM bytes per launch of this kernel variant from the committed counter summary,
    if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash():
        return None
    entry = rec.get("per_variant", {}).get(str(variant))
    return entry.get("hbm_bytes_per_launch") if entry else None


def cpu_baseline(inst, alpha, budget_s: float):
    """The oracle's closed form (as it stands) on the host cores, repeated up to ~budget_s."""
    from oracle import qbvm_oracle as O
    d, m, n = inst.d, inst.m, inst.n
    runs = 0
    t0 = time.perf_counter()
    c0 = time.process_time()
    while True:
        O.closed_form(inst.g_delta, d, m, n, inst.L, inst.T, alpha, O.PQ)
        runs += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    value = runs * n * m ** d / wall / 1e6
    return {"value": round(value, 3), "unit": "Munknowns/s", "cores": max(1, round(cpu / wall)),
            "kind": "oracle",
            "sample": f"{runs} full closed-form solves of the same 2D m={m} n={n} instance "
                      f"(orthonormal DST-I via scipy, per-mode formula, all {n + 1} levels), {wall:.1f} s"}


def solve_3d_bench(steps: int):
    """3D m=127, n=128, T=0.5, alpha=1e-5 full solve (2.1 GB output): time and per-kernel rooflines."""
    import torch

    from paper_2107_06381_amd import qbvm, workloads as W

    inst = W.config_3d()
    dev = torch.device("cuda:0")
    g = torch.from_numpy(inst.g_delta).to(dev)
    plan = qbvm.Plan(3, 127, 128, 1.0, 0.5)
    tune = plan.autotune()
    y = torch.empty((129, 127, 127, 127), dtype=torch.float64, device=dev)
    for _ in range(2):
        plan.solve(1e-5, qbvm.QBVM_PQ, g, y)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.solve(1e-5, qbvm.QBVM_PQ, g, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    qbvm.profile_reset()
    qbvm.profile_enable(True)
    for _ in range(steps):
        plan.solve(1e-5, qbvm.QBVM_PQ, g, y)
    torch.cuda.synchronize()
    rep = qbvm.profile_report()
    qbvm.profile_enable(False)
    kernels = {k: {"launches_per_step": r["launches"] / steps, "avg_us": round(r["total_ms"] / r["launches"] * 1e3, 1),
                   "hbm_frac": round(r["bytes"] / (r["total_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
               for k, r in rep.items()}
    step_bytes = sum(v["bytes"] for v in rep.values()) / steps
    del y
    plan.close()
    torch.cuda.empty_cache()
    unk = 128 * 127 ** 3
    return {"workload": "3D PinT-QBVM, m=127 (7-point), n=128 (N_t=129), T=0.5, alpha=1e-5, Gaussian bump, 0.1% noise",
            "ms_per_solve": round(ms, 4), "Munknowns_per_s": round(unk / (ms * 1e-3) / 1e6, 1),
            "step_hbm_roofline_frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernels": kernels, "autotune": tune}


def alpha_choice_bench(train_count: int, test_count: int, lat_count: int, steps: int):
    """Learned vs bisection alpha choice on 2D m=127, n=128, T=1 (noise 0.1%..5%)."""
    import numpy as np
    import torch

    from paper_2107_06381_amd import alpha_model as AM, qbvm

    plan = qbvm.Plan(2, 127, 128, 1.0, 1.0)
    t0 = time.perf_counter()
    train_ds = AM.make_dataset(plan, seed=4, count=train_count)
    t_label = time.perf_counter() - t0
    t0 = time.perf_counter()
    model, hist = AM.train(train_ds, steps=steps, batch=256, lr=3e-3, log_every=steps)
    t_train = time.perf_counter() - t0
    del train_ds
    test_ds = AM.make_dataset(plan, seed=5, count=test_count, keep_z0=True)
    plan.set_alpha_model(model.blob())
    idx = np.arange(test_count)
    AM.choose_all(plan, test_ds, idx[:20], use_learned=True)  # warm-up
    AM.choose_all(plan, test_ds, idx[:20], use_learned=False)
    a_l, lat_l, fb = AM.choose_all(plan, test_ds, idx, use_learned=True)
    li = idx[:lat_count]
    a_b, lat_b, _ = AM.choose_all(plan, test_ds, li, use_learned=False)
    e_l = AM.reconstruction_errors(plan, test_ds, a_l, idx)
    e_dp = AM.reconstruction_errors(plan, test_ds, test_ds.alpha_dp, idx)
    e_prior = AM.reconstruction_errors(plan, test_ds, test_ds.delta, idx)
    ok = test_ds.hits == 0
    r = e_l[ok] / e_dp[ok]
    return {
        "workload": f"2D m=127 n=128 T=1, {train_count} training / {test_count} held-out instances, "
                    "labels: 30-step discrepancy bisection (tau=1.1) on [1e-20, 1]",
        "label_gen_s": round(t_label, 2), "train_s": round(t_train, 2), "train_steps": steps,
        "final_train_mse_std": round(hist[-1][1], 6) if hist else None,
        "error_ratio_learned_over_dp": {"mean": round(float(r.mean()), 5), "median": round(float(np.median(r)), 5),
                                        "p95": round(float(np.quantile(r, 0.95)), 5)},
        "error_ratio_alpha_eq_delta_over_dp": round(float(np.mean(e_prior[ok] / e_dp[ok])), 4),
        "fallback_rate": round(float(fb.mean()), 4),
        "latency_us": {"learned_mean": round(float(lat_l.mean() * 1e6), 1),
                       "learned_median": round(float(np.median(lat_l) * 1e6), 1),
                       "bisection_mean": round(float(lat_b.mean() * 1e6), 1),
                       "bisection_median": round(float(np.median(lat_b) * 1e6), 1),
                       "speedup_median": round(float(np.median(lat_b) / np.median(lat_l)), 2),
                       "bisection_sample": int(lat_count)},
    }


def batched_bench(reps: int = 3):
    """512 uneven 1D/2D instances: one batched graph launch vs 512 qbvm_solve calls."""
    import numpy as np
    import torch

    from paper_2107_06381_amd import qbvm, workloads as W

    dev = torch.device("cuda:0")
    insts = W.config_batched()
    grids = [(i.d, i.m, i.n, i.L, i.T) for i in insts]
    alphas = [i.alpha for i in insts]
    variants = [0] * len(insts)
    gs = [torch.from_numpy(i.g_delta).to(dev) for i in insts]
    ys = [torch.empty((i.n + 1,) + (i.m,) * i.d, dtype=torch.float64, device=dev) for i in insts]
    t0 = time.perf_counter()
    plans = {}
    for gr in grids:
        if gr not in plans:
            plans[gr] = qbvm.Plan(*gr)
    t_plans = time.perf_counter() - t0

    def seq(sel):
        for k in sel:
            plans[grids[k]].solve(alphas[k], 0, gs[k], ys[k])

    def bat(sel):
        qbvm.solve_batched([grids[k] for k in sel], [alphas[k] for k in sel], [0] * len(sel),
                           [gs[k] for k in sel], [ys[k] for k in sel])

    def timed(fn, sel):
        best = 1e30
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn(sel)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        return best

    classes = {"all": list(range(len(insts))),
               "1d": [k for k in range(len(insts)) if grids[k][0] == 1],
               "2d_small": [k for k in range(len(insts)) if grids[k][0] == 2 and grids[k][1] < 160],
               "2d_large": [k for k in range(len(insts)) if grids[k][0] == 2 and grids[k][1] >= 160]}
    out = {}
    t0 = time.perf_counter()
    for name, sel in classes.items():
        bat(sel)  # builds and caches the graph for this set
        seq(sel)
    t_graph = time.perf_counter() - t0
    for name, sel in classes.items():
        ts = timed(seq, sel)
        tb = timed(bat, sel)
        unk = sum(grids[k][2] * grids[k][1] ** grids[k][0] for k in sel)
        out[name] = {"instances": len(sel), "sequential_ms": round(ts * 1e3, 3), "batched_ms": round(tb * 1e3, 3),
                     "speedup": round(ts / tb, 3), "batched_Munknowns_per_s": round(unk / tb / 1e6, 1)}
    # sampled parity of the batched output
    from oracle import qbvm_oracle as O
    errs = []
    bat(classes["all"])
    torch.cuda.synchronize()
    for k in [0, 1, 255, 256, 300, 511]:
        i = insts[k]
        lv = [0, i.n]
        yc = O.closed_form(i.g_delta, i.d, i.m, i.n, i.L, i.T, i.alpha, 0, levels=lv)
        yk = ys[k][lv].cpu().numpy()
        errs.append(max(float(np.linalg.norm(yk[j] - yc[j]) / np.linalg.norm(yc[j])) for j in range(2)))
    qbvm.batched_cache_clear()
    return {"workload": "512 instances: 256 1D m in [63,1023] + 256 2D m in [63,255], n in [64,512], "
                        "alpha in [1e-6,1e-1], noise 0.1%..5%, every level output",
            "plan_build_s": round(t_plans, 2), "graph_build_s": round(t_graph, 2),
            "timing": "host clock around the enqueue and the final synchronize, best of %d" % reps,
            "classes": out, "sampled_parity_max_rel_err": max(errs)}


def general_rhs_bench(steps: int = 20):
    """General right-hand side (every level nonzero) on the 2D workload's grid: seconds per
    solve through qbvm_solve_general, and the HBM fraction of its schedule (d sine passes
    in, the time kernel, d passes out: 16 B per unknown each)."""
    import numpy as np
    import torch
    from paper_2107_06381_amd import qbvm
    d, m, n, alpha = 2, 255, 256, 1e-4
    plan = qbvm.Plan(d, m, n, 1.0, 1.0)
    plan.autotune()
    f = torch.from_numpy(np.random.default_rng(11).standard_normal((n + 1, m, m))).to("cuda:0")
    y = torch.empty_like(f)
    for _ in range(3):
        plan.solve_general(alpha, qbvm.QBVM_PQ, f, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.solve_general(alpha, qbvm.QBVM_PQ, f, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    unknowns = n * m ** d
    sched_bytes = 16.0 * (n + 1) * m ** d * (2 * d + 1)
    plan.close()
    return {"workload": "2D m=255, n=256 (N_t=257), general right-hand side (all 257 levels), alpha=1e-4",
            "ms_per_solve": round(ms, 4), "Munknowns_per_s": round(unknowns / (ms * 1e-3) / 1e6, 1),
            "schedule_bytes_per_unknown": 16 * (2 * d + 1),
            "step_hbm_roofline_frac": round(sched_bytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}


def operator_1d_bench(steps: int = 20):
    """1D solve with a variable-coefficient operator -(kappa u')' in place of -Lap_h
    (Step (b) as a complex Thomas solve per shift) on the largest 1D grid: seconds per
    solve and the kernel split."""
    import numpy as np
    import torch
    from paper_2107_06381_amd import qbvm, workloads as W
    m, n, alpha = 2047, 4095, 1e-4
    rng = np.random.default_rng(17)
    lo, di, up = W.diffusion_operator_1d(m, rng)
    plan = qbvm.Plan(1, m, n, 1.0, 1.0)
    plan.set_operator_1d(lo, di, up)
    g = torch.from_numpy(rng.standard_normal(m)).to("cuda:0")
    y = torch.empty((n + 1, m), dtype=torch.float64, device="cuda:0")
    for _ in range(3):
        plan.solve(alpha, qbvm.QBVM_PQ, g, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.solve(alpha, qbvm.QBVM_PQ, g, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    qbvm.profile_reset()
    qbvm.profile_enable(True)
    for _ in range(5):
        plan.solve(alpha, qbvm.QBVM_PQ, g, y)
    torch.cuda.synchronize()
    rep = qbvm.profile_report()
    qbvm.profile_enable(False)
    plan.close()
    kernels = {k: {"avg_us": round(r["total_ms"] / r["launches"] * 1e3, 1),
                   "GBps": round(r["bytes"] / (r["total_ms"] * 1e-3) / 1e9, 1)} for k, r in rep.items()}
    # the 1D configuration (m=127, n=128, Dirichlet stencil): latency of one solve
    inst = W.config_1d()
    p1 = qbvm.Plan(1, inst.m, inst.n, inst.L, inst.T)
    g1 = torch.from_numpy(inst.g_delta).to("cuda:0")
    y1 = torch.empty((inst.n + 1, inst.m), dtype=torch.float64, device="cuda:0")
    for _ in range(5):
        p1.solve(inst.alpha, qbvm.QBVM_PQ, g1, y1)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(100):
        p1.solve(inst.alpha, qbvm.QBVM_PQ, g1, y1)
    e1.record()
    torch.cuda.synchronize()
    us1 = e0.elapsed_time(e1) / 100 * 1e3
    p1.close()
    return {"workload": "1D m=2047, n=4095 (N_t=4096), variable kappa (contrast 4), alpha=1e-4, every level",
            "ms_per_solve": round(ms, 4), "Munknowns_per_s": round(n * m / (ms * 1e-3) / 1e6, 1),
            "kernels": kernels,
            "config_1d_m127_n128_us_per_solve": round(us1, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-alpha", action="store_true", help="skip the learned/bisection alpha-choice section")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-instance batched section")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D solve section")
    ap.add_argument("--no-general", action="store_true", help="skip the general right-hand-side section")
    ap.add_argument("--no-operator", action="store_true", help="skip the 1D variable-coefficient section")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (reference kernel for counter calibration)")
    ap.add_argument("--alpha-train", type=int, default=20000)
    ap.add_argument("--alpha-test", type=int, default=2000)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2107_06381_amd import qbvm, workloads as W

    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    d, m, n, alpha = 2, 255, 256, 1e-4
    inst = W.config_2d()
    dev = torch.device("cuda:0")
    g = torch.from_numpy(inst.g_delta).to(dev)
    plan = qbvm.Plan(d, m, n, 1.0, 1.0)
    tune = plan.autotune()  # kernel-variant choice, excluded from the timed region
    y = torch.empty((n + 1, m, m), dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        plan.solve(alpha, qbvm.QBVM_PQ, g, y)
    torch.cuda.synchronize()

    # timed region: K solves on the current stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        plan.solve(alpha, qbvm.QBVM_PQ, g, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    unknowns = n * m ** d
    value = unknowns / (ms * 1e-3) / 1e6

    # parity of the benchmarked output on sampled levels (the oracle is test
    # infrastructure; only the CPU-baseline leg and this sample check call it)
    parity = None
    cpu = None
    if not args.no_cpu:
        from oracle import qbvm_oracle as O
        levels = [0, n // 2, n]
        yc = O.closed_form(inst.g_delta, d, m, n, 1.0, 1.0, alpha, O.PQ, levels=levels)
        yl = y[levels].cpu().numpy()
        parity = float(max(np.linalg.norm(yl[i] - yc[i]) / np.linalg.norm(yc[i]) for i in range(3)))
        cpu = cpu_baseline(inst, alpha, args.cpu_budget)

    # per-kernel durations: HIP events around each launch on the plan's stream
    qbvm.profile_reset()
    qbvm.profile_enable(True)
    for _ in range(args.steps):
        plan.solve(alpha, qbvm.QBVM_PQ, g, y)
    torch.cuda.synchronize()
    rep = qbvm.profile_report()
    qbvm.profile_enable(False)
    kernels = {}
    for k, r in rep.items():
        avg_ms = r["total_ms"] / r["launches"]
        kernels[k] = {"launches_per_step": r["launches"] / args.steps, "avg_us": round(avg_ms * 1e3, 2),
                      "GBps": round(r["bytes"] / (r["total_ms"] * 1e-3) / 1e9, 1),
                      "TFLOPs": round(r["flops"] / (r["total_ms"] * 1e-3) / 1e12, 2)}
    dom = max(rep, key=lambda k: rep[k]["total_ms"])
    r = rep[dom]
    avg_s = r["total_ms"] / r["launches"] * 1e-3
    bytes_per_launch = r["bytes"] / r["launches"]
    achieved = bytes_per_launch / avg_s / 1e9
    workload = "2d_m255_n256"
    role_variant = {"dst_rows": "rows", "dst_cols": "cols", "time_spectral": "time"}.get(dom)
    traffic = read_traffic(dom, workload, tune["variants"][role_variant]) if role_variant else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_us": round(avg_s * 1e6, 2)}
    step_bytes = sum(v["bytes"] for v in rep.values()) / args.steps
    del y
    torch.cuda.empty_cache()
    solve3d = None if args.no_3d else solve_3d_bench(5)
    alpha = None if args.no_alpha else alpha_choice_bench(args.alpha_train, args.alpha_test, 200, 3000)
    batched = None if args.no_batched else batched_bench()
    general = None if args.no_general else general_rhs_bench()
    operator_1d = None if args.no_operator else operator_1d_bench()
    line = {
        "metric": "PinT solve Munknowns/s (n*m^d, FP64)",
        "value": round(value, 2),
        "unit": "Munknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D PinT-QBVM all-at-once solve, m=255 (5-point), n=256 (N_t=257), T=1, "
                               "alpha=1e-4, 64 random sine modes, 0.5% noise, every level output",
                   "unknowns_n_md": unknowns, "unknowns_true": (n + 1) * m ** d},
        "roofline": roofline,
        "step_hbm_roofline_frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernels": kernels,
        "autotune": tune,
        "solve_3d": solve3d,
        "alpha_choice": alpha,
        "batched": batched,
        "general_rhs": general,
        "operator_1d": operator_1d,
        "parity_rel_err": parity,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
