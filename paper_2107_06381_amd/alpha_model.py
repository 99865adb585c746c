"""Learned choice of the regularisation parameter (an addition, not from the paper).

The paper fixes alpha a priori (alpha = delta, or tau*delta for PinT-MQBVM,
Section 5).  Here a small network predicts log10(alpha) from the sine spectrum of
g_delta and the noise level; the label is the discrepancy-principle alpha found
by bisection (D(alpha) = 1.1 delta), which also stays the fallback whenever a
prediction misses the discrepancy window.

Everything numerical runs in the library: labels by qbvm_bisect_batched,
features by qbvm_features, training by qbvm_mlp_loss_grad and qbvm_adam_step,
selection by qbvm_choose_alpha (qbvm_choose_alpha_each for timed sweeps).  The host only generates the synthetic data,
shuffles minibatch order and computes the 33 feature means/standard deviations.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from . import qbvm
from . import workloads as W

D_IN, D_H = 33, 64
NPARAM = qbvm.MLP_PARAMS


def init_params(rng: np.random.Generator) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) in the layout W1|b1|W2|b2|W3|b3."""
    parts = []
    for shape, fan in [((D_H, D_IN), D_IN), ((D_H,), D_IN), ((D_H, D_H), D_H), ((D_H,), D_H), ((D_H,), D_H),
                       ((1,), D_H)]:
        a = 1.0 / math.sqrt(fan)
        parts.append(rng.uniform(-a, a, size=shape).ravel())
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == NPARAM
    return p


@dataclasses.dataclass
class AlphaModel:
    params: np.ndarray      # NPARAM float32
    feat_mean: np.ndarray   # 33
    feat_std: np.ndarray    # 33
    y_mean: float
    y_std: float

    def blob(self) -> np.ndarray:
        return np.concatenate([self.params.astype(np.float32), self.feat_mean.astype(np.float32),
                               self.feat_std.astype(np.float32),
                               np.array([self.y_mean, self.y_std], dtype=np.float32)])

    def save(self, path: str):
        np.save(path, self.blob())

    @staticmethod
    def load(path: str) -> "AlphaModel":
        b = np.load(path, allow_pickle=False).astype(np.float32)
        if b.size != qbvm.MODEL_FLOATS:
            raise ValueError("not a model blob")
        return AlphaModel(b[:NPARAM].copy(), b[NPARAM:NPARAM + 33].copy(), b[NPARAM + 33:NPARAM + 66].copy(),
                          float(b[NPARAM + 66]), float(b[NPARAM + 67]))


@dataclasses.dataclass
class Dataset:
    feats: "object"        # torch float32 (count, 33) on the GPU
    alpha_dp: np.ndarray   # float64 (count,)
    hits: np.ndarray       # int32 (count,)
    delta: np.ndarray      # float64 (count,)
    g_delta: "object"      # torch float64 (count, m, m) on the GPU (kept for evaluation)
    z0: Optional[np.ndarray]


def make_dataset(plan: qbvm.Plan, seed: int, count: int, chunk: int = 2048, keep_z0: bool = False,
                 opts: Optional[qbvm.AlphaOpts] = None) -> Dataset:
    """Synthetic 2D instances (random lowest sine modes, noise 0.1%..5%), labelled by
    the batched discrepancy bisection and turned into features, all on the GPU."""
    import torch
    gd, deltas, z0, _ = W.config_learned(seed, count, m=plan.m, n=plan.n, T=plan.T)
    dev = torch.device("cuda", torch.cuda.current_device())
    G = torch.from_numpy(gd).to(dev)
    Dl = torch.from_numpy(deltas).to(dev)
    feats = torch.empty((count, D_IN), dtype=torch.float32, device=dev)
    alphas = np.empty(count)
    hits = np.empty(count, dtype=np.int32)
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        a, h = plan.bisect_batched(qbvm.QBVM_PQ, G[s:e], Dl[s:e], opts)
        feats[s:e] = plan.features(G[s:e], Dl[s:e])
        alphas[s:e] = a.cpu().numpy()
        hits[s:e] = h.cpu().numpy()
    return Dataset(feats, alphas, hits, deltas, G, z0 if keep_z0 else None)


def train(ds: Dataset, steps: int = 3000, batch: int = 256, lr: float = 2e-3, seed: int = 0,
          log_every: int = 0) -> tuple[AlphaModel, list]:
    """Adam on the mean-squared error of standardised log10(alpha_DP), on the GPU."""
    import torch
    dev = ds.feats.device
    ok = ds.hits == 0
    Xh = ds.feats.cpu().numpy()[ok].astype(np.float64)
    yh = np.log10(ds.alpha_dp[ok])
    fm = Xh.mean(0)
    fs = Xh.std(0)
    fs[fs < 1e-6] = 1.0
    ym, ys = float(yh.mean()), float(yh.std() if yh.std() > 0 else 1.0)
    Xs = ((Xh - fm) / fs).astype(np.float32)
    Ys = ((yh - ym) / ys).astype(np.float32)
    rng = np.random.default_rng(seed)
    P = torch.from_numpy(init_params(rng)).to(dev)
    Mo = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
    Vo = torch.zeros(NPARAM, dtype=torch.float32, device=dev)
    grad = torch.empty(NPARAM, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    n = Xs.shape[0]
    batch = min(batch, n)
    per_epoch = max(1, n // batch)
    hist = []
    step = 0
    while step < steps:
        perm = rng.permutation(n)
        Xd = torch.from_numpy(np.ascontiguousarray(Xs[perm])).to(dev)
        Yd = torch.from_numpy(np.ascontiguousarray(Ys[perm])).to(dev)
        for b in range(per_epoch):
            if step >= steps:
                break
            sl = slice(b * batch, (b + 1) * batch)
            qbvm.mlp_loss_grad(P, Xd[sl], Yd[sl], grad, loss)
            step += 1
            qbvm.adam_step(P, grad, Mo, Vo, step, lr * (0.5 * (1 + math.cos(math.pi * step / steps)) * 0.95 + 0.05))
            if log_every and step % log_every == 0:
                hist.append((step, float(loss)))
    torch.cuda.synchronize()
    model = AlphaModel(P.cpu().numpy(), fm.astype(np.float32), fs.astype(np.float32), ym, ys)
    return model, hist


def predict_log10(model: AlphaModel, feats) -> np.ndarray:
    """Network output on the GPU (qbvm_mlp_forward), de-standardised."""
    import torch
    dev = feats.device
    X = ((feats.cpu().numpy().astype(np.float64) - model.feat_mean) / model.feat_std).astype(np.float32)
    P = torch.from_numpy(model.params).to(dev)
    out = qbvm.mlp_forward(P, torch.from_numpy(X).to(dev))
    return out.cpu().numpy().astype(np.float64) * model.y_std + model.y_mean


def reconstruction_errors(plan: qbvm.Plan, ds: Dataset, alphas: np.ndarray, idx) -> np.ndarray:
    """e_h = ||y^0(alpha) - z0||_h (Section 5) for the instances idx, y^0 by qbvm_solve
    (the difference and its norm are taken on the GPU)."""
    import torch
    h = plan.Lx / (plan.m + 1)
    dev = ds.g_delta.device
    out = np.empty(len(idx))
    y0 = torch.empty((plan.m,) * plan.d, dtype=torch.float64, device=dev)
    for i, k in enumerate(idx):
        plan.solve(float(alphas[i]), qbvm.QBVM_PQ, ds.g_delta[k], y0, output=qbvm.OUT_Y0)
        z = torch.from_numpy(ds.z0[k]).to(dev)
        out[i] = h ** (plan.d / 2) * float(torch.linalg.vector_norm(y0 - z))
    return out


def error_curve(plan: qbvm.Plan, ds: Dataset, idx, grid) -> np.ndarray:
    """e_h(alpha) for every alpha of `grid` (rows: instances idx, columns: grid)."""
    return np.stack([reconstruction_errors(plan, ds, np.full(len(idx), float(a)), idx) for a in grid], 1)


def choose_all(plan: qbvm.Plan, ds: Dataset, idx, use_learned: bool, win=(1.05, 1.15)):
    """qbvm_choose_alpha_each over the instances idx (batch size 1 each): alphas, per-call
    latencies (seconds, measured in the library around each synchronous call), fallback flags."""
    import torch
    opts = qbvm.default_alpha_opts(use_learned)
    opts.win_lo, opts.win_hi = win
    idx = np.asarray(idx, dtype=np.int64)
    G = ds.g_delta.index_select(0, torch.from_numpy(idx).to(ds.g_delta.device)).contiguous()
    torch.cuda.synchronize()
    alphas, infos, lat = plan.choose_alpha_each(qbvm.QBVM_PQ, G, ds.delta[idx], opts)
    return alphas, lat, infos["used_fallback"].astype(bool)
