"""The paper's PinT error tables reproduced with the GPU solver (Section 5).

Example 2 (Table 2, 2D) and Example 1 (Table 1, 1D): the same data, noise model and
a-priori alpha as the oracle pins in test_oracle_pins.py, solved through the C ABI.
Each solution is checked against the oracle on the same noisy data (relative 1e-8).
With alpha = delta (PinT-QBVM) and alpha = tau*delta (PinT-MQBVM) the two methods solve
the same system (PM(alpha) = PQ(alpha/tau), the remark after Theorem 4.1), so the
paper's PQ and PM entries of one mesh and noise level differ only by their noise
draw, which is unknown.  The reconstruction error e_h = ||y^0 - z0||_h is therefore
checked against the band between the two printed values, widened by 12% (Table 2,
eps = 1e-3 and 1e-4, where the regularisation bias dominates) or 30% (Table 1, noise
dominated); the GPU solves of both variants are checked to agree.
"""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from oracle import qbvm_oracle as O  # noqa: E402
from paper_2107_06381_amd import qbvm  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _table(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            rows[(tok[0], int(tok[1]))] = [float(v) for v in tok[3:7]]
    return rows


def _paper_noise(g, eps, rng):
    return g * (1.0 + eps * rng.uniform(-1.0, 1.0, g.shape))


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _in_band(e, name, M, col, tol):
    t = _table(name)
    lo, hi = sorted((t[("PQ", M)][col], t[("PM", M)][col]))
    return lo * (1 - tol) <= e <= hi * (1 + tol), (lo, hi)


@pytest.mark.parametrize("method,M", [(m, M) for M in (16, 32, 64, 128) for m in ("PQ", "PM")])
def test_table2_on_gpu(method, M):
    L, T, m, n = math.pi, 1.0, M - 1, M
    h = L / M
    x = h * np.arange(1, M)
    X2, X1 = np.meshgrid(x, x, indexing="ij")
    z0 = np.sin(X1) * np.sin(X2)
    g = math.exp(-2 * T) * z0
    rng = np.random.default_rng(2021)
    variant = qbvm.QBVM_PQ if method == "PQ" else qbvm.QBVM_PM
    plan = qbvm.Plan(2, m, n, L, T)
    for col, eps in [(0, 1e-1), (1, 1e-2), (2, 1e-3), (3, 1e-4)]:
        errs = []
        for _ in range(3):
            gd = _paper_noise(g, eps, rng)
            delta = h * np.linalg.norm(gd - g)
            alpha = delta if variant == qbvm.QBVM_PQ else (T / n) * delta
            gdev = torch.from_numpy(gd).to(DEV)
            y0 = plan.solve(alpha, variant, gdev, output=qbvm.OUT_Y0)
            other = qbvm.QBVM_PM if variant == qbvm.QBVM_PQ else qbvm.QBVM_PQ
            y0o = plan.solve(alpha * (T / n) if other == qbvm.QBVM_PM else alpha * n / T, other, gdev,
                             output=qbvm.OUT_Y0)
            torch.cuda.synchronize()
            y0 = y0.cpu().numpy()
            assert _rel(y0o.cpu().numpy(), y0) < 1e-12
            yo = O.closed_form(gd, 2, m, n, L, T, alpha, variant, levels=[0])[0]
            assert _rel(y0, yo) < 1e-8
            errs.append(O.reconstruction_error(y0, z0, L))
        e = float(np.mean(errs))
        ok, band = _in_band(e, "table2_pint_errors.txt", M, col, 0.12)
        say(f"Table 2 {method} M={M} eps={eps:g}: e_h GPU {e:.3f}, paper PQ/PM {band[0]:.3f}..{band[1]:.3f}")
        if eps <= 1e-3:
            assert ok, (method, M, eps, e, band)
    plan.close()


@pytest.mark.parametrize("method,M", [(m, M) for M in (256, 512, 1024) for m in ("PQ", "PM")])
def test_table1_on_gpu(method, M):
    L, T = math.pi, 1.0
    m, n = M - 1, M
    h = L / M
    x = h * np.arange(1, M)
    z0 = np.where(x <= math.pi / 2, 2 * x, 2 * (math.pi - x))
    k = np.arange(1, 200, 2)
    zT = 8 / math.pi * np.sum(np.cos(k[:, None] * (2 * x[None, :] - math.pi) / 2) / k[:, None] ** 2
                              * np.exp(-k[:, None] ** 2 * T), 0)
    rng = np.random.default_rng(2107 + M)
    variant = qbvm.QBVM_PQ if method == "PQ" else qbvm.QBVM_PM
    plan = qbvm.Plan(1, m, n, L, T)
    for col, eps in enumerate([1e-1, 1e-2, 1e-3, 1e-4]):
        errs = []
        for _ in range(6):
            gd = _paper_noise(zT, eps, rng)
            delta = math.sqrt(h) * np.linalg.norm(gd - zT)
            alpha = delta if variant == qbvm.QBVM_PQ else (T / n) * delta
            y = plan.solve(alpha, variant, torch.from_numpy(gd).to(DEV))
            torch.cuda.synchronize()
            y = y.cpu().numpy()
            yo = O.closed_form(gd, 1, m, n, L, T, alpha, variant, levels=[0, n])
            assert _rel(y[0], yo[0]) < 1e-8
            errs.append(O.reconstruction_error(y[0], z0, L))
        e = float(np.mean(errs))
        ok, band = _in_band(e, "table1_pint_errors.txt", M, col, 0.30)
        say(f"Table 1 {method} M={M} eps={eps:g}: e_h GPU {e:.3f}, paper PQ/PM {band[0]:.3f}..{band[1]:.3f}")
        assert ok, (method, M, eps, e, band)
    plan.close()
