"""Benchmark of the PinT-QBVM all-at-once solve on one MI355X.

Headline workload (the largest single-GPU configuration): 3D, Omega=(0,1)^3, m=127
interior points per dimension (7-point Laplacian), n=128 backward-Euler steps
(N_t = 129), T=0.5, alpha=1e-5, PinT-QBVM, FP64; initial datum = Gaussian bump
(centre (0.4,0.5,0.6), width 0.1), 0.1% relative Gaussian noise (seeded,
synthetic).  One step = one full solve (every level: 129 levels of 127^3 values,
2.1 GB), inputs resident in HBM.  Metric: solve throughput in Munknowns/s on the
n*m^d basis.  Side sections: the 2D workload (m=255, n=256), alpha choice,
batched solves, general right-hand side, 1D/2D/3D variable-coefficient operators.

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


# sources that no recorded counter summary depends on (the operator-path Krylov kernels)
HASH_EXCLUDE = {"qbvm_krylov.hip", "qbvm_bodies_krylov.hpp"}


def source_hash() -> str:
    """Hash of the kernel and executor sources the committed counter summaries were taken on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2107_06381_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f in HASH_EXCLUDE:
            continue
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


def cpu_share() -> int:
    """Host threads this process may use (its affinity mask, at most 16: one GPU's share of the box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    return "unknown"


def cpu_baseline(inst, alpha, budget_s: float):
    """The oracle's closed form (as it stands: orthonormal DST-I by scipy.fft, the per-mode
    formula, every level) on the host cores, repeated until ~budget_s has passed."""
    import scipy.fft

    from oracle import qbvm_oracle as O
    d, m, n = inst.d, inst.m, inst.n
    workers = cpu_share()
    runs = 0
    t0 = time.perf_counter()
    with scipy.fft.set_workers(workers):
        while True:
            O.closed_form(inst.g_delta, d, m, n, inst.L, inst.T, alpha, O.PQ)
            runs += 1
            if time.perf_counter() - t0 >= budget_s:
                break
    wall = time.perf_counter() - t0
    value = runs * n * m ** d / wall / 1e6
    return {"value": round(value, 3), "unit": "Munknowns/s", "cores": workers, "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "sample": f"{runs} full closed-form solves of the {d}D m={m} n={n} workload instance (orthonormal "
                      f"DST-I via scipy.fft with workers={workers}, per-mode formula, all {n + 1} levels), "
                      f"{wall:.1f} s"}


def copy_ceiling_gbps(numel: int, reps: int = 5) -> float:
    """Plain device-to-device copy of an FP64 array of this size: bytes read + written per second."""
    import torch
    src = torch.ones(numel, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = 1e30
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(reps):
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * 8.0 * numel / best / 1e9


ROLE_OF_KERNEL = {"dst_rows": "rows", "dst_cols": "cols", "time_spectral": "time"}


def solve_bench(inst, steps: int, warmup: int, tag: str, parity_levels=None):
    """Time `steps` full solves (every level) of one workload instance on the current stream,
    then the per-kernel durations (HIP events around each launch on the plan's stream) and the
    roofline of the kernel with the largest share of time."""
    import numpy as np
    import torch

    from paper_2107_06381_amd import qbvm

    d, m, n = inst.d, inst.m, inst.n
    dev = torch.device("cuda:0")
    g = torch.from_numpy(inst.g_delta).to(dev)
    plan = qbvm.Plan(d, m, n, inst.L, inst.T)
    tune = plan.autotune()  # kernel-variant choice, excluded from the timed region
    y = torch.empty((n + 1,) + (m,) * d, dtype=torch.float64, device=dev)
    for _ in range(warmup):
        plan.solve(inst.alpha, qbvm.QBVM_PQ, g, y)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.solve(inst.alpha, qbvm.QBVM_PQ, g, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    parity = None
    if parity_levels is not None:
        from oracle import qbvm_oracle as O
        yc = O.closed_form(inst.g_delta, d, m, n, inst.L, inst.T, inst.alpha, O.PQ, levels=parity_levels)
        yl = y[parity_levels].cpu().numpy()
        parity = float(max(np.linalg.norm(yl[i] - yc[i]) / np.linalg.norm(yc[i])
                           for i in range(len(parity_levels))))
    qbvm.profile_reset()
    qbvm.profile_enable(True)
    for _ in range(steps):
        plan.solve(inst.alpha, qbvm.QBVM_PQ, g, y)
    torch.cuda.synchronize()
    rep = qbvm.profile_report()
    qbvm.profile_enable(False)
    kernels = {}
    for k, r in rep.items():
        avg_ms = r["total_ms"] / r["launches"]
        kernels[k] = {"launches_per_step": r["launches"] / steps, "avg_us": round(avg_ms * 1e3, 2),
                      "GBps": round(r["bytes"] / (r["total_ms"] * 1e-3) / 1e9, 1),
                      "TFLOPs": round(r["flops"] / (r["total_ms"] * 1e-3) / 1e12, 2)}
    dom = max(rep, key=lambda k: rep[k]["total_ms"])
    r = rep[dom]
    avg_s = r["total_ms"] / r["launches"] * 1e-3
    bytes_per_launch = r["bytes"] / r["launches"]
    achieved = bytes_per_launch / avg_s / 1e9
    role = ROLE_OF_KERNEL.get(dom)
    var = tune["plane_variant"] if dom == "dst_plane" else (tune["variants"][role] if role else None)
    traffic = read_traffic(dom, tag, var) if var is not None else None
    step_bytes = sum(v["bytes"] for v in rep.values()) / steps
    numel = y.numel()
    del y
    plan.close()
    torch.cuda.empty_cache()
    copy = copy_ceiling_gbps(numel)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_us": round(avg_s * 1e6, 2),
                "launch_timing": "HIP events around each launch on the plan's stream",
                "copy_ceiling_GBps": round(copy, 1), "frac_of_copy": round(achieved / copy, 4)}
    return {"ms": ms, "value": n * m ** d / (ms * 1e-3) / 1e6, "kernels": kernels, "roofline": roofline,
            "step_hbm_roofline_frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "step_bytes_per_unknown": round(step_bytes / ((n + 1) * m ** d), 2),
            "autotune": tune, "parity_rel_err": parity}


ALPHA_GRID_LOG10 = [x / 4.0 for x in range(-64, 1)]  # 1e-16 .. 1, four points per decade


def alpha_config_bench(T: float, train_count: int, test_count: int, steps: int, grid_count: int):
    """Learned vs bisection alpha choice on 2D m=127, n=128 at final time T (noise 0.1%..5%):
    labels, training, then on the held-out set the reconstruction error of the learned alpha,
    of alpha_DP and of the paper's a-priori alpha = delta, the error over a grid of alpha on
    `grid_count` held-out instances, and per-call latencies of both modes on every held-out
    instance (timed in the library)."""
    import numpy as np

    from paper_2107_06381_amd import alpha_model as AM, qbvm

    plan = qbvm.Plan(2, 127, 128, 1.0, T)
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
    a_b, lat_b, _ = AM.choose_all(plan, test_ds, idx, use_learned=False)
    e_l = AM.reconstruction_errors(plan, test_ds, a_l, idx)
    e_dp = AM.reconstruction_errors(plan, test_ds, test_ds.alpha_dp, idx)
    e_prior = AM.reconstruction_errors(plan, test_ds, test_ds.delta, idx)
    ok = test_ds.hits == 0
    r = e_l[ok] / e_dp[ok]
    rp = e_prior[ok] / e_dp[ok]
    gi = idx[ok][:grid_count]
    grid = [10.0 ** g for g in ALPHA_GRID_LOG10]
    curve = AM.error_curve(plan, test_ds, gi, grid) / e_dp[gi][:, None]
    med = np.median(curve, 0)
    band = [ALPHA_GRID_LOG10[i] for i in range(len(grid)) if med[i] <= 1.05]
    plan.close()
    return {
        "workload": f"2D m=127 n=128 T={T}, {train_count} training / {test_count} held-out instances, "
                    "labels: 30-step discrepancy bisection (tau=1.1) on [1e-20, 1]",
        "label_gen_s": round(t_label, 2), "train_s": round(t_train, 2), "train_steps": steps,
        "final_train_mse_std": round(hist[-1][1], 6) if hist else None,
        "alpha_dp_log10_median": round(float(np.median(np.log10(test_ds.alpha_dp[ok]))), 3),
        "error_ratio_learned_over_dp": {"mean": round(float(r.mean()), 5), "median": round(float(np.median(r)), 5),
                                        "p95": round(float(np.quantile(r, 0.95)), 5)},
        "error_ratio_alpha_eq_delta_over_dp": {"mean": round(float(rp.mean()), 4),
                                               "median": round(float(np.median(rp)), 4)},
        "error_curve": {"instances": int(len(gi)), "log10_alpha": ALPHA_GRID_LOG10,
                        "median_ratio_to_dp": [round(float(x), 4) for x in med],
                        "best_grid_ratio_median": round(float(np.median(curve.min(1))), 4),
                        "log10_alpha_within_5pct": [min(band), max(band)] if band else None},
        "fallback_rate": round(float(fb.mean()), 4),
        "latency_us": {"learned_mean": round(float(lat_l.mean() * 1e6), 1),
                       "learned_median": round(float(np.median(lat_l) * 1e6), 1),
                       "bisection_mean": round(float(lat_b.mean() * 1e6), 1),
                       "bisection_median": round(float(np.median(lat_b) * 1e6), 1),
                       "speedup_median": round(float(np.median(lat_b) / np.median(lat_l)), 2),
                       "instances": int(test_count),
                       "timing": "steady clock around each qbvm_choose_alpha call inside qbvm_choose_alpha_each"},
    }


def alpha_choice_bench(train_count: int, test_count: int, steps: int):
    """The learned-alpha workload (T=1) and the same family at T=0.1, where the error has a
    pronounced minimum in alpha (the T=1 error curve is flat over several decades)."""
    return {"T1": alpha_config_bench(1.0, train_count, test_count, steps, 400),
            "T0.1": alpha_config_bench(0.1, train_count, test_count, steps, 400)}


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


def operator_diffusion_bench(d: int = 2, reps: int = 3):
    """2D or 3D solve with the variable-coefficient operator -div(kappa grad u) (Step (b) by
    batched preconditioned conjugate orthogonal CG over the shifts) on the 2D workload's
    grid (m=255, n=256) or the 3D workload's grid (m=127, n=128): seconds per solve
    (synchronous; host clock, best of reps), iterations, the kernel split, and the HBM
    fraction of the iteration's algorithmic bytes."""
    import numpy as np
    import torch
    from paper_2107_06381_amd import qbvm, workloads as W
    m, n, alpha, tol = (255, 256, 1e-4, 1e-12) if d == 2 else (127, 128, 1e-5, 1e-12)
    rng = np.random.default_rng(19)
    kap = W.diffusion_coefficients_2d(m, rng) if d == 2 else W.diffusion_coefficients_3d(m, rng)
    plan = qbvm.Plan(d, m, n, 1.0, 1.0 if d == 2 else 0.5)
    plan.autotune()
    if d == 2:
        plan.set_operator_2d(*kap, tol, 200)
    else:
        plan.set_operator_3d(*kap, tol, 200)
    g = torch.from_numpy(rng.standard_normal((m,) * d)).to("cuda:0")
    y = torch.empty((n + 1,) + (m,) * d, dtype=torch.float64, device="cuda:0")
    plan.solve(alpha, qbvm.QBVM_PQ, g, y)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        plan.solve(alpha, qbvm.QBVM_PQ, g, y)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    st = plan.operator_stats()
    qbvm.profile_reset()
    qbvm.profile_enable(True)
    plan.solve(alpha, qbvm.QBVM_PQ, g, y)
    torch.cuda.synchronize()
    rep = qbvm.profile_report()
    qbvm.profile_enable(False)
    plan.close()
    kernels = {k: {"launches": r["launches"], "avg_us": round(r["total_ms"] / r["launches"] * 1e3, 1),
                   "GBps": round(r["bytes"] / (r["total_ms"] * 1e-3) / 1e9, 1)} for k, r in rep.items()}
    tot_bytes = sum(r["bytes"] for r in rep.values())
    tot_ms = sum(r["total_ms"] for r in rep.values())
    H = (n + 2) // 2
    work = ("2D m=255, n=256 (N_t=257), alpha=1e-4" if d == 2 else "3D m=127, n=128 (N_t=129), T=0.5, alpha=1e-5")
    return {"workload": f"{work}, -div(kappa grad u), kappa log-smooth contrast 4, COCG tol 1e-12, every level",
            "ms_per_solve": round(best * 1e3, 3), "Munknowns_per_s": round(n * m ** d / best / 1e6, 1),
            "iterations": st["iterations"], "max_rel_residual": st["max_rel_residual"],
            "shifted_systems": H, "iteration_bytes_per_complex_unknown": 320,
            "kernel_ms_sum": round(tot_ms, 3),
            "kernels_hbm_frac": round(tot_bytes / (tot_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "kernels": kernels}


# kernels of each benchmarked workload: sine-transform length and the time kernel's symbol prefix
TRAFFIC_WORKLOADS = {
    "3d_m127_n128": {"sine_n": 256, "time_prefix": "k_time_gt<3, 43,", "title": "3D PinT-QBVM solve, m=127, n=128 (N_t=129)",
                     "flags": "--no-2d"},
    "2d_m255_n256": {"sine_n": 512, "time_prefix": "k_time_p2<256,", "title": "2D PinT-QBVM solve, m=255, n=256 (N_t=257)",
                     "flags": ""},
}


def _read_pmc(directory: str, counter: str):
    """{dispatch id: (kernel name, counter value)} from the rocprofv3 counter CSVs under directory."""
    import csv
    import glob
    out = {}
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {directory}")
    for path in files:
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                key = (path, row["Dispatch_Id"])
                name, val = out.get(key, (row["Kernel_Name"], 0.0))
                out[key] = (name, val + float(row["Counter_Value"]))
    return out


def _kernel_role(name: str, w: dict):
    """(role, variant) of a solve kernel of workload w from its symbol, else None."""
    import re
    n = w["sine_n"]
    mm = re.search(r"k_dst_(rows|cols)_p2<(\d+), (\d+)", name)
    if mm and int(mm.group(2)) == n:
        var = int(mm.group(3))
        if var == 2 and ("rows" in mm.group(1) or "false" in name):
            return ("dst_input", var)
        return ("dst_" + mm.group(1), var)
    mm = re.search(r"k_dst_plane_p2<(\d+), (\d+)>", name)
    if mm and int(mm.group(1)) == n:
        return ("dst_plane", int(mm.group(2)))
    if w["time_prefix"] in name:
        mm = re.search(r"k_time_(?:gt<\d+, \d+|p2<\d+), (\d+)", name)
        if mm:
            return ("time_spectral", int(mm.group(1)))
    return None


def write_traffic_summary(fetch_dir: str, write_dir: str, tag: str, out_dir: str = None):
    """Scale FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what they read for the 1 GiB
    reference copy of --copy-probe and write profiles/<role>_<tag>_traffic.json (bytes per
    launch per kernel variant, keyed to the current kernel sources) and a Markdown table."""
    import statistics
    w = TRAFFIC_WORKLOADS[tag]
    fetch = _read_pmc(fetch_dir, "FETCH_SIZE")
    write = _read_pmc(write_dir, "WRITE_SIZE")
    gib_kib = float(1 << 20)

    def copy_kib(rec):
        # the reference copies are the first three copy dispatches of the run (--copy-probe runs first)
        ids = sorted((k for k, (nm, _) in rec.items() if "copy" in nm.lower()), key=lambda k: (k[0], int(k[1])))
        vals = [rec[k][1] for k in ids[:3]]
        if not vals:
            raise SystemExit("reference copy not found: run the profiled command with --copy-probe")
        return statistics.median(vals)

    fscale = gib_kib / copy_kib(fetch)
    wscale = gib_kib / copy_kib(write)

    def per_kernel(rec):
        d = {}
        for nm, v in rec.values():
            d.setdefault(nm, []).append(v)
        return d

    fk, wk = per_kernel(fetch), per_kernel(write)
    roles = {}
    rows = []
    for nm in sorted(set(fk) & set(wk)):
        rv = _kernel_role(nm, w)
        if rv is None:
            continue
        role, var = rv
        fm, wm = statistics.median(fk[nm]), statistics.median(wk[nm])
        hbm = (fm * fscale + wm * wscale) * 1024.0
        roles.setdefault(role, {})[str(var)] = {"kernel": nm, "dispatches": len(fk[nm]), "fetch_kib_median": fm,
                                                "write_kib_median": wm, "hbm_bytes_per_launch": round(hbm)}
        rows.append((nm, role, len(fk[nm]), fm, wm, fm * fscale * 1024 / 1e6, wm * wscale * 1024 / 1e6))
    prof = out_dir or os.path.join(ROOT, "profiles")
    cmd = ("rocprofv3 --pmc {c} --output-format csv -d <{d}> -o {o} -- python3 bench.py --steps 3 --warmup 1 "
           "--no-cpu {flags} --no-alpha --no-batched --no-general --no-operator --copy-probe")
    cmds = [cmd.format(c="FETCH_SIZE", d="fetch_dir", o="fetch", flags=w["flags"]).replace("  ", " "),
            cmd.format(c="WRITE_SIZE", d="write_dir", o="write", flags=w["flags"]).replace("  ", " "),
            f"python3 bench.py --traffic-summary <fetch_dir> <write_dir> {tag}"]
    for role, per in roles.items():
        with open(os.path.join(prof, f"{role}_{tag}_traffic.json"), "w") as f:
            json.dump({"source_hash": source_hash(), "fetch_scale": fscale, "write_scale": wscale,
                       "per_variant": per, "commands": cmds}, f, indent=1)
    with open(os.path.join(prof, f"traffic_{tag}.md"), "w") as f:
        f.write(f"# HBM traffic per launch: {w['title']}\n\n")
        f.write("Commands (repository root, one MI355X; `cd /tmp && export TMPDIR=/tmp` first for the profiler):\n\n")
        for c in cmds:
            f.write(f"    {c}\n")
        f.write(f"\n`--copy-probe` first runs a plain 1 GiB device-to-device copy three times, the reference "
                f"kernel; its counters give the scale factors {fscale:.3f} (FETCH_SIZE) and {wscale:.3f} (WRITE_SIZE).  Median over the "
                f"dispatches of each kernel (the autotuner runs every variant; the kept one has the most "
                f"dispatches).  Kernel sources hash {source_hash()}.\n\n")
        f.write("| kernel | role | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled MB read | scaled MB written |\n")
        f.write("|---|---|---|---|---|---|---|\n")
        for nm, role, nd, fm, wm, rmb, wmb in rows:
            f.write(f"| `{nm}` | {role} | {nd} | {fm:.0f} | {wm:.0f} | {rmb:.1f} | {wmb:.1f} |\n")
    print(f"wrote {len(roles)} traffic records for {tag}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D solve section")
    ap.add_argument("--no-alpha", action="store_true", help="skip the learned/bisection alpha-choice section")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-instance batched section")
    ap.add_argument("--no-general", action="store_true", help="skip the general right-hand-side section")
    ap.add_argument("--no-operator", action="store_true", help="skip the 1D, 2D and 3D variable-coefficient sections")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (reference kernel for counter calibration)")
    ap.add_argument("--alpha-train", type=int, default=20000)
    ap.add_argument("--alpha-test", type=int, default=2000)
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "WORKLOAD"),
                    help="write profiles/<kernel>_<WORKLOAD>_traffic.json from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of this script with --copy-probe, then exit")
    args = ap.parse_args()
    if args.traffic_summary:
        write_traffic_summary(*args.traffic_summary)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2107_06381_amd import workloads as W

    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    # headline: the largest single-GPU workload, 3D m=127, n=128 (N_t=129), T=0.5, alpha=1e-5
    inst = W.config_3d()
    head = solve_bench(inst, args.steps, args.warmup, "3d_m127_n128",
                       parity_levels=None if args.no_cpu else [0, 1, 64, 128])
    cpu = None if args.no_cpu else cpu_baseline(inst, inst.alpha, args.cpu_budget)
    del inst
    solve2d = None
    if not args.no_2d:
        i2 = W.config_2d()
        r2 = solve_bench(i2, args.steps, args.warmup, "2d_m255_n256",
                         parity_levels=None if args.no_cpu else [0, 128, 256])
        solve2d = {"workload": "2D PinT-QBVM, m=255 (5-point), n=256 (N_t=257), T=1, alpha=1e-4, "
                               "64 random sine modes, 0.5% noise, every level output",
                   "ms_per_solve": round(r2["ms"], 5), "Munknowns_per_s": round(r2["value"], 1),
                   "roofline": r2["roofline"], "step_hbm_roofline_frac": r2["step_hbm_roofline_frac"],
                   "step_bytes_per_unknown": r2["step_bytes_per_unknown"], "kernels": r2["kernels"],
                   "autotune": r2["autotune"], "parity_rel_err": r2["parity_rel_err"]}
    alpha = None if args.no_alpha else alpha_choice_bench(args.alpha_train, args.alpha_test, 3000)
    batched = None if args.no_batched else batched_bench()
    general = None if args.no_general else general_rhs_bench()
    operator_1d = None if args.no_operator else operator_1d_bench()
    operator_2d = None if args.no_operator else operator_diffusion_bench(2)
    operator_3d = None if args.no_operator else operator_diffusion_bench(3, reps=2)
    n, m = 128, 127
    line = {
        "metric": "PinT solve Munknowns/s (n*m^d, FP64)",
        "value": round(head["value"], 2),
        "unit": "Munknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D PinT-QBVM all-at-once solve, m=127 (7-point), n=128 (N_t=129), T=0.5, "
                               "alpha=1e-5, Gaussian bump, 0.1% noise, every level output",
                   "unknowns_n_md": n * m ** 3, "unknowns_true": (n + 1) * m ** 3},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "step_hbm_roofline_frac": head["step_hbm_roofline_frac"],
        "step_bytes_per_unknown": head["step_bytes_per_unknown"],
        "kernels": head["kernels"],
        "autotune": head["autotune"],
        "parity_rel_err": head["parity_rel_err"],
        "solve_2d": solve2d,
        "alpha_choice": alpha,
        "batched": batched,
        "general_rhs": general,
        "operator_1d": operator_1d,
        "operator_2d": operator_2d,
        "operator_3d": operator_3d,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
