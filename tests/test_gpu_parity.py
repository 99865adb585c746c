"""GPU parity: the HIP library (through its C ABI) against the CPU FP64 oracle.

Tolerance: relative 2-norm 1e-8 on the full solution and, separately, on y^0 and
y^N (the bar the design targets); measured errors are ~1e-13.
"""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from oracle import qbvm_oracle as O  # noqa: E402
from oracle import mlp_oracle as M  # noqa: E402
from paper_2107_06381_amd import qbvm, workloads as W  # noqa: E402
from tests.parity_util import level_ok, omega_abs  # noqa: E402

TOL = 1e-8
DEV = torch.device("cuda:0")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def gpu_solve(d, m, n, L, T, alpha, variant, g, output=qbvm.OUT_ALL):
    p = qbvm.Plan(d, m, n, L, T)
    y = p.solve(alpha, variant, to_dev(g), output=output)
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    p.close()
    return out


CASES = [
    # d, m, n, alpha, variant  (prime / composite / Rader / Bluestein lengths, ragged tiles)
    (1, 7, 6, 1e-2, 0), (1, 127, 128, 1e-3, 0), (1, 33, 40, 1e-6, 1), (1, 64, 63, 1e-6, 0),
    (1, 1, 1, 0.5, 0), (1, 300, 211, 1e-4, 0), (1, 1023, 512, 1e-5, 0),
    (2, 1, 1, 0.5, 0), (2, 5, 4, 1e-3, 0), (2, 15, 16, 1e-4, 1), (2, 20, 11, 1e-2, 0),
    (2, 31, 100, 1e-8, 0), (2, 63, 256, 1e-4, 0), (2, 100, 52, 1e-6, 1), (2, 47, 129, 1e-12, 0),
    (3, 4, 5, 1e-3, 0), (3, 9, 8, 1e-5, 1), (3, 31, 42, 1e-3, 0),
    # power-of-two kernels: N_t = 64, 128, 256, 257 (Rader), sine lengths 64 .. 2048
    (2, 63, 63, 1e-4, 0), (3, 15, 127, 1e-3, 1), (2, 20, 255, 1e-6, 0), (2, 33, 256, 1e-4, 0),
    (2, 255, 6, 1e-3, 0), (2, 511, 3, 1e-2, 1), (2, 1023, 2, 1e-3, 0), (3, 63, 64, 1e-4, 0),
    # padded level pipeline: 2D N_t = 256, 3D N_t = 64, 2D m = 511 with N_t = 128
    (2, 63, 255, 1e-5, 1), (3, 31, 63, 1e-3, 0), (2, 511, 127, 1e-4, 0),
    # the ends of the bisection bracket (alpha = 1e-20 .. 1), both variants
    (2, 63, 64, 1e-20, 0), (2, 63, 64, 1.0, 1), (1, 127, 128, 1e-20, 1), (3, 15, 16, 1e-20, 0),
    (2, 255, 256, 1e-20, 0), (2, 255, 256, 1.0, 0),
]


@pytest.mark.parametrize("d,m,n,alpha,variant", CASES)
def test_solve_vs_oracle(d, m, n, alpha, variant):
    say(f"[case] d={d} m={m} n={n} alpha={alpha} variant={variant}")
    L, T = 1.0, 0.9
    g = np.random.default_rng(d * 1000 + m * 7 + n).standard_normal((m,) * d)
    y = gpu_solve(d, m, n, L, T, alpha, variant, g)
    yc = O.closed_form(g, d, m, n, L, T, alpha, variant)
    assert np.all(np.isfinite(y))
    assert rel(y, yc) < TOL
    assert rel(y[0], yc[0]) < TOL
    ok, r = level_ok(y[-1], yc[-1], yc[0], n, n + 1, omega_abs(alpha, variant, T / n))
    assert ok, r


@pytest.mark.parametrize("d,m,n,alpha,variant", [(1, 31, 30, 1e-3, 0), (2, 12, 10, 1e-5, 1), (2, 5, 6, 1e-1, 0)])
def test_solve_vs_sparse_lu(d, m, n, alpha, variant):
    """Against the assembled all-at-once system solved by SuperLU (no structure used)."""
    say(f"[case] splu d={d} m={m} n={n}")
    g = np.random.default_rng(3).standard_normal((m,) * d)
    y = gpu_solve(d, m, n, 1.0, 1.0, alpha, variant, g)
    ys = O.solve_splu(g, d, m, n, 1.0, 1.0, alpha, variant)
    assert rel(y, ys) < TOL and rel(y[0], ys[0]) < TOL and rel(y[-1], ys[-1]) < TOL


def test_config_1d_full():
    """1D, m=127, n=128, alpha=1e-3, 1% noise: against SuperLU of the all-at-once system."""
    say("[case] config 1d")
    inst = W.config_1d()
    y = gpu_solve(1, 127, 128, 1.0, 1.0, 1e-3, 0, inst.g_delta)
    ys = O.solve_splu(inst.g_delta, 1, 127, 128, 1.0, 1.0, 1e-3, O.PQ)
    assert rel(y, ys) < TOL and rel(y[0], ys[0]) < TOL and rel(y[-1], ys[-1]) < TOL
    assert O.residual(y, inst.g_delta, 1, 127, 128, 1.0, 1.0, 1e-3, O.PQ) < 1e-11


def test_config_2d_full():
    """2D, m=255, n=256 (N_t = 257, prime), alpha=1e-4, in the kernel variants the autotuner
    keeps (the bench's launch configuration): every level against the closed form."""
    say("[case] config 2d")
    inst = W.config_2d()
    p = qbvm.Plan(2, 255, 256, 1.0, 1.0)
    say("variants", p.autotune()["variants"])
    y = p.solve(1e-4, 0, to_dev(inst.g_delta))
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    p.close()
    yc = O.closed_form(inst.g_delta, 2, 255, 256, 1.0, 1.0, 1e-4, O.PQ)
    assert rel(y, yc) < TOL and rel(y[0], yc[0]) < TOL and rel(y[-1], yc[-1]) < TOL
    # sampled levels against the all-at-once rows (residual of levels 1..n)
    assert O.residual(y, inst.g_delta, 2, 255, 256, 1.0, 1.0, 1e-4, O.PQ) < 1e-8


def test_config_3d_every_level():
    """3D, m=127, n=128, T=0.5, alpha=1e-5 (2.1 GB output), autotuned variants (the bench's launch
    configuration): every level against the closed form, in chunks of 16 levels."""
    import scipy.fft
    say("[case] config 3d, every level")
    inst = W.config_3d()
    m, n = 127, 128
    p = qbvm.Plan(3, m, n, 1.0, 0.5)
    tune = p.autotune()
    say("variants", tune["variants"], "plane pass", tune["plane_variant"], tune["ms_separate_x2_x1"], tune["ms_plane_v012"])
    y = p.solve(1e-5, 0, to_dev(inst.g_delta))
    torch.cuda.synchronize()
    assert bool(torch.isfinite(y).all())
    # the other schedules (separate x_2 and x_1 passes, every plane-pass variant): same
    # values to rounding
    for v in [-1, 0, 1, 2]:
        p.set_plane(v >= 0, max(v, 0))
        y2 = p.solve(1e-5, 0, to_dev(inst.g_delta))
        torch.cuda.synchronize()
        diff = float(torch.linalg.vector_norm(y2 - y) / torch.linalg.vector_norm(y))
        say("schedule", v, "vs autotuned", diff)
        assert diff < 1e-13
        del y2
    p.close()
    worst = 0.0
    with scipy.fft.set_workers(min(16, len(os.sched_getaffinity(0)))):
        for c0 in range(0, n + 1, 16):
            levels = list(range(c0, min(n + 1, c0 + 16)))
            yl = y[levels].cpu().numpy()
            yc = O.closed_form(inst.g_delta, 3, m, n, 1.0, 0.5, 1e-5, O.PQ, levels=levels)
            for i, t in enumerate(levels):
                e = rel(yl[i], yc[i])
                worst = max(worst, e)
                assert e < TOL, (t, e)
    say("worst level rel err", worst)
    del y


@pytest.mark.parametrize("n,alpha,variant,pv", [(128, 1e-4, 0, 0), (127, 1e-2, 1, 1), (63, 1e-6, 0, 2)])
def test_plane_pass_2d_vs_oracle(n, alpha, variant, pv):
    """2D m = 127 (sine length 256): the plane pass does both sine transforms of each level;
    every level against the closed form, with plane-pass variant pv and with the separate passes."""
    say(f"[case] plane pass 2d m=127 n={n} variant {pv}")
    m = 127
    g = np.random.default_rng(n).standard_normal((m, m))
    p = qbvm.Plan(2, m, n, 1.0, 1.0)
    p.set_plane(True, pv)
    assert p.plane_variant() == pv
    y = p.solve(alpha, variant, to_dev(g)).cpu().numpy()
    p.set_plane(False)
    assert not p.uses_plane()
    y2 = p.solve(alpha, variant, to_dev(g)).cpu().numpy()
    p.close()
    yc = O.closed_form(g, 2, m, n, 1.0, 1.0, alpha, variant)
    w = omega_abs(alpha, variant, 1.0 / n)
    for yy in (y, y2):
        assert rel(yy, yc) < TOL
        for t in range(n + 1):
            ok, e = level_ok(yy[t], yc[t], yc[0], t, n + 1, w)
            assert ok, (t, e)


def test_plane_pass_refused_where_unsupported():
    p = qbvm.Plan(2, 63, 64, 1.0, 1.0)
    assert not p.uses_plane()
    with pytest.raises(qbvm.QbvmError) as e:
        p.set_plane(True)
    assert e.value.code == -5
    p.close()


@pytest.mark.parametrize("d,m,n,levels", [
    (1, 2047, 4095, [0, 1, 2048, 4095]),   # 1D: largest m and N_t = 4096
    (2, 2047, 1, None),                    # 2D: sine length 4096
    (2, 63, 2047, [0, 1, 1024, 2047]),     # 2D: N_t = 2048
    (3, 511, 1, None),                     # 3D: 2.1 GB per level array pair
])
def test_maximum_sizes(d, m, n, levels):
    """The largest grids the ABI accepts, against the closed form on the listed levels."""
    say(f"[case] max size d={d} m={m} n={n}")
    g = np.random.default_rng(d * 31 + m).standard_normal((m,) * d)
    p = qbvm.Plan(d, m, n)
    y = p.solve(1e-4, 0, to_dev(g))
    torch.cuda.synchronize()
    lv = list(range(n + 1)) if levels is None else levels
    yl = y[lv].cpu().numpy()
    assert bool(torch.isfinite(y).all())
    del y
    p.close()
    torch.cuda.empty_cache()
    yc = O.closed_form(g, d, m, n, 1.0, 1.0, 1e-4, O.PQ, levels=lv)
    for i, t in enumerate(lv):
        ok, r = level_ok(yl[i], yc[i], yc[0], t, n + 1, omega_abs(1e-4, 0, 1.0 / n))
        assert rel(yl[i], yc[i]) < TOL or ok, (t, r)


@pytest.mark.parametrize("d,m,n", [(1, 50, 33), (2, 40, 31), (3, 10, 12)])
def test_single_level_outputs(d, m, n):
    say(f"[case] out modes d={d}")
    g = np.random.default_rng(4).standard_normal((m,) * d)
    for out, lev in [(qbvm.OUT_Y0, 0), (qbvm.OUT_YN, n)]:
        y = gpu_solve(d, m, n, 1.0, 1.0, 1e-4, 0, g, output=out)
        yc = O.closed_form(g, d, m, n, 1.0, 1.0, 1e-4, O.PQ, levels=[lev])[0]
        assert rel(y, yc) < TOL


@pytest.mark.parametrize("d,m,n,alpha,variant", [(1, 127, 128, 1e-3, 0), (2, 63, 64, 1e-4, 1), (2, 100, 52, 1e-6, 0),
                                                 (3, 15, 16, 1e-3, 0), (2, 255, 256, 1e-4, 0), (1, 1, 1, 0.5, 0),
                                                 (3, 127, 128, 1e-5, 0)])
def test_general_rhs_vs_oracle(d, m, n, alpha, variant):
    """General right-hand side in every block row (source terms / preconditioner use)."""
    say(f"[case] general rhs d={d} m={m} n={n}")
    f = np.random.default_rng(d * 17 + m + n).standard_normal((n + 1,) + (m,) * d)
    p = qbvm.Plan(d, m, n, 1.0, 0.9)
    y = p.solve_general(alpha, variant, to_dev(f))
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    p.close()
    yc = O.closed_form_general(f, d, m, n, 1.0, 0.9, alpha, variant)
    assert np.all(np.isfinite(y))
    assert rel(y, yc) < TOL and rel(y[0], yc[0]) < TOL
    if m ** d * (n + 1) < 20000:
        ys = O.solve_general_splu(f, d, m, n, 1.0, 0.9, alpha, variant)
        assert rel(y, ys) < TOL


@pytest.mark.parametrize("m,n", [(127, 128), (255, 256)])
def test_general_rhs_rank_one_and_in_place(m, n):
    """f = (f0, 0, ..., 0) reproduces qbvm_solve; y may be f itself (generic kernels at
    N_t = 129, the padded pipeline at N_t = 257)."""
    say(f"[case] general rhs rank one m={m} n={n}")
    d, alpha = 2, 1e-4
    g = np.random.default_rng(8).standard_normal((m, m))
    p = qbvm.Plan(d, m, n)
    f = O.rhs_allatonce(g, n, alpha, O.PQ, 1.0).reshape((n + 1, m, m))
    fd = to_dev(f)
    y1 = p.solve(alpha, 0, to_dev(g)).clone()
    p.solve_general(alpha, 0, fd, fd)  # in place
    torch.cuda.synchronize()
    assert rel(fd.cpu().numpy(), y1.cpu().numpy()) < 1e-11


@pytest.mark.parametrize("d,m", [(3, 31), (2, 127)])
def test_good_thomas_variants(d, m):
    """N_t = 129 = 3 * 43: the Good-Thomas time kernel's four variants (direct 43-point rows
    or Rader's algorithm on the 42-point prime-factor DFT, two output chunkings), selected by
    hand, against the closed form, every level."""
    n, alpha = 128, 1e-4
    say(f"[case] good-thomas variants d={d} m={m}")
    g = np.random.default_rng(31).standard_normal((m,) * d)
    yc = O.closed_form(g, d, m, n, 1.0, 0.5, alpha, O.PQ)
    p = qbvm.Plan(d, m, n, 1.0, 0.5)
    gd = to_dev(g)
    ys = []
    for V in range(4):
        p.set_variants(time=V)
        y = p.solve(alpha, qbvm.QBVM_PQ, gd).cpu().numpy()
        ys.append(y)
        assert rel(y, yc) < TOL, (V, rel(y, yc))
        w = omega_abs(alpha, 0, 0.5 / n)
        ok, r = level_ok(y[-1], yc[-1], yc[0], n, n + 1, w)
        assert ok, (V, r)
    assert rel(ys[2], ys[0]) < 1e-12 and rel(ys[3], ys[1]) < 1e-12
    with pytest.raises(qbvm.QbvmError):
        p.set_variants(time=4)
    p.close()


@pytest.mark.parametrize("d,m,n", [(2, 255, 256), (3, 63, 63)])
def test_every_kernel_variant(d, m, n):
    """Every sine-pass, time and general-time kernel variant, selected by hand, against
    the oracle (the autotuner keeps one per role; the others must be right too)."""
    say(f"[case] every variant d={d} m={m} n={n}")
    rng = np.random.default_rng(21)
    g = rng.standard_normal((m,) * d)
    f = rng.standard_normal((n + 1,) + (m,) * d)
    alpha = 1e-4
    p = qbvm.Plan(d, m, n)
    base = p.variants()
    yc = O.closed_form(g, d, m, n, 1.0, 1.0, alpha, O.PQ)
    ygc = O.closed_form_general(f, d, m, n, 1.0, 1.0, alpha, O.PQ)
    gd, fd = to_dev(g), to_dev(f)
    y = torch.empty((n + 1,) + (m,) * d, dtype=torch.float64, device="cuda:0")

    def check(rhs_general, **kw):
        p.set_variants(**kw)
        assert all(p.variants()[k] == v for k, v in kw.items())
        if rhs_general:
            p.solve_general(alpha, qbvm.QBVM_PQ, fd, y)
        else:
            p.solve(alpha, qbvm.QBVM_PQ, gd, y)
        torch.cuda.synchronize()
        e = rel(y.cpu().numpy(), ygc if rhs_general else yc)
        p.set_variants(**base)
        assert e < TOL, (kw, e)

    for V in range(8):
        check(False, rows=V)
        check(False, cols=V)
        check(True, rows=V, cols=V)
    for V in range(6):
        check(False, time=V)
        check(True, general=V)
    for bad in (dict(rows=8), dict(cols=-2), dict(time=6), dict(general=6)):
        with pytest.raises(qbvm.QbvmError):
            p.set_variants(**bad)
    assert p.variants() == base
    p.close()
    q = qbvm.Plan(2, 20, 11)  # generic kernels only
    with pytest.raises(qbvm.QbvmError):
        q.set_variants(rows=0)
    q.set_variants()
    q.close()


@pytest.mark.parametrize("m,n,alpha,variant,adv", [(127, 128, 1e-3, 0, 0.0), (1000, 511, 1e-5, 1, 0.0),
                                                   (2047, 4095, 1e-4, 0, 2.0), (1, 1, 0.5, 0, 0.0),
                                                   (255, 256, 1e-6, 0, 0.0)])
def test_operator_1d_vs_oracle(m, n, alpha, variant, adv):
    """1D solve with a tridiagonal spatial operator in place of -Lap_h (variable kappa,
    upwinded advection), every level and the single-level outputs, against the oracle's
    eigenbasis closed form; clearing the operator restores the Dirichlet stencil."""
    say(f"[case] operator 1d m={m} n={n} adv={adv}")
    rng = np.random.default_rng(m + 3 * n)
    lo, di, up = W.diffusion_operator_1d(m, rng, advection=adv)
    g = rng.standard_normal(m)
    A = O.tridiagonal_matrix(lo, di, up)
    yc = O.closed_form_operator(g, A, n, 0.6, alpha, variant)
    p = qbvm.Plan(1, m, n, 1.0, 0.6)
    p.set_operator_1d(lo, di, up)
    gd = to_dev(g)
    y = p.solve(alpha, variant, gd)
    y0 = p.solve(alpha, variant, gd, output=qbvm.OUT_Y0)
    yn = p.solve(alpha, variant, gd, output=qbvm.OUT_YN)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), yc) < TOL
    assert rel(y0.cpu().numpy(), yc[0]) < TOL and rel(yn.cpu().numpy(), yc[-1]) < TOL
    if m * (n + 1) < 40000:
        ys = O.solve_splu_operator(g, A, n, 0.6, alpha, variant)
        assert rel(y.cpu().numpy(), ys) < TOL
    with pytest.raises(qbvm.QbvmError):
        p.discrepancy(alpha, variant, gd)
    p.set_operator_1d()
    y = p.solve(alpha, variant, gd)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), O.closed_form(g, 1, m, n, 1.0, 0.6, alpha, variant)) < TOL
    p.close()


@pytest.mark.parametrize("m", [1251, 1400])
def test_1d_long_bluestein_sine_lengths(m):
    """1D m = 1251 (2(m+1) = 8 * 313) and 1400 (2 * 3 * 467): sine lengths whose plain
    Bluestein core (2N - 1 points and more) exceeds 4096; the symmetric form of the sine
    kernel needs P >= N - 1, here 4096.  The solve (tridiagonal path, every output mode) and
    the discrepancy, which works in the sine basis, match the oracle."""
    say(f"[case] 1d long bluestein sine m={m}")
    n, alpha = 106, 1e-4
    g = np.random.default_rng(12).standard_normal(m)
    p = qbvm.Plan(1, m, n, 1.0, 0.8)
    gd = to_dev(g)
    y = p.solve(alpha, 0, gd)
    yn = p.solve(alpha, 0, gd, output=qbvm.OUT_YN)
    torch.cuda.synchronize()
    yc = O.closed_form(g, 1, m, n, 1.0, 0.8, alpha, O.PQ)
    assert rel(y.cpu().numpy(), yc) < TOL and rel(yn.cpu().numpy(), yc[-1]) < TOL
    D = p.discrepancy(alpha, 0, gd)
    Do = O.discrepancy(alpha, g, 1, m, n, 1.0, 0.8)
    assert abs(D / Do - 1.0) < 1e-10
    p.close()


@pytest.mark.parametrize("d,m,n", [(2, 10, 7), (2, 22, 9), (3, 22, 5), (2, 52, 11), (2, 100, 6),
                                   (2, 178, 20), (2, 400, 3), (2, 600, 2), (2, 1251, 2)])
def test_bluestein_sine_cores(d, m, n):
    """Sine lengths N = 2(m+1) with a prime factor above 7 take the Bluestein sine passes on
    the power-of-two engine (symmetric form, P >= N - 1); these grids use every core from
    64 (2D and 3D) to 4096, every level compared with the closed form."""
    say(f"[case] bluestein sine d={d} m={m} n={n}")
    alpha = 1e-4
    g = np.random.default_rng(m + d).standard_normal((m,) * d)
    p = qbvm.Plan(d, m, n, 1.0, 1.0)
    y = p.solve(alpha, 0, to_dev(g))
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), O.closed_form(g, d, m, n, 1.0, 1.0, alpha, O.PQ)) < TOL
    p.close()


def test_operator_rejected_off_1d():
    say("[case] operator on a 2D plan")
    p = qbvm.Plan(2, 15, 8)
    with pytest.raises(qbvm.QbvmError):
        p.set_operator_1d(np.ones(14), np.ones(15), np.ones(14))
    p.close()


def test_pq_pm_identity_and_determinism():
    """PinT-MQBVM with alpha equals PinT-QBVM with alpha/tau (Section 4); repeated solves are bitwise equal."""
    say("[case] identity")
    d, m, n = 2, 33, 40
    tau = 1.0 / n
    g = to_dev(np.random.default_rng(5).standard_normal((m, m)))
    p = qbvm.Plan(d, m, n)
    ym = p.solve(1e-6, qbvm.QBVM_PM, g).clone()
    yq = p.solve(1e-6 / tau, qbvm.QBVM_PQ, g).clone()
    ym2 = p.solve(1e-6, qbvm.QBVM_PM, g).clone()
    torch.cuda.synchronize()
    assert rel(ym.cpu().numpy(), yq.cpu().numpy()) < 1e-12
    assert torch.equal(ym, ym2)


def test_invalid_arguments():
    p = qbvm.Plan(1, 8, 8)
    g = torch.zeros(8, dtype=torch.float64, device=DEV)
    for a in [0.0, -1.0, float("nan"), float("inf")]:
        with pytest.raises(qbvm.QbvmError) as e:
            p.solve(a, 0, g)
        assert e.value.code == -1
    with pytest.raises(qbvm.QbvmError):
        p.solve(1e-3, 7, g)
    with pytest.raises(ValueError):
        p.solve(1e-3, 0, torch.zeros(9, dtype=torch.float64, device=DEV))


# ---------------------------------------------------------------- discrepancy / bisection
def test_discrepancy_vs_oracle():
    say("[case] discrepancy")
    inst = W.sine_mode_instance(2, 63, 64, 1.0, 0.0, 0.01, np.random.default_rng(6))
    p = qbvm.Plan(2, 63, 64)
    g = to_dev(inst.g_delta)
    for a in [1e-14, 1e-10, 1e-6, 1e-2]:
        Dg = p.discrepancy(a, 0, g)
        Do = O.discrepancy(a, inst.g_delta, 2, 63, 64, 1.0, 1.0)
        assert abs(Dg - Do) <= 1e-9 * Do


def test_choose_alpha_bisection_vs_oracle():
    say("[case] bisection")
    inst = W.sine_mode_instance(2, 127, 128, 1.0, 0.0, 0.01, np.random.default_rng(7))
    p = qbvm.Plan(2, 127, 128)
    a, info = p.choose_alpha(0, to_dev(inst.g_delta), inst.delta)
    ao, hit = O.bisect_alpha(inst.g_delta, inst.delta, 2, 127, 128, 1.0, 1.0)
    assert hit == 0 and info.bracket_hit == 0
    # both bisect the same bracket; decisions agree except within rounding of D near the root
    assert abs(math.log10(a) - math.log10(ao)) < 1e-6
    assert abs(info.discrepancy / (1.1 * inst.delta) - 1.0) < 1e-5
    assert info.iterations == 33


def test_bisect_batched_matches_single():
    say("[case] bisect batched")
    rng = np.random.default_rng(8)
    insts = [W.sine_mode_instance(2, 31, 32, 1.0, 0.0, eps, rng) for eps in [0.002, 0.01, 0.03, 0.05, 1e-9]]
    p = qbvm.Plan(2, 31, 32)
    G = to_dev(np.stack([i.g_delta for i in insts]))
    Dl = to_dev(np.array([i.delta for i in insts]))
    alphas, hits = p.bisect_batched(0, G, Dl)
    torch.cuda.synchronize()
    for k, inst in enumerate(insts):
        ao, hit = O.bisect_alpha(inst.g_delta, inst.delta, 2, 31, 32, 1.0, 1.0)
        assert int(hits[k]) == hit
        assert abs(math.log10(float(alphas[k])) - math.log10(ao)) < 1e-6


def test_features_vs_oracle():
    say("[case] features")
    gd, deltas, _, _ = W.config_learned(11, 6, m=127, n=128)
    p = qbvm.Plan(2, 127, 128)
    f = p.features(to_dev(gd), to_dev(deltas)).cpu().numpy()
    for i in range(6):
        fo = O.features(gd[i], deltas[i])
        np.testing.assert_allclose(f[i], fo.astype(np.float32), rtol=2e-6, atol=2e-5)


# ---------------------------------------------------------------- network kernels
def test_mlp_forward_and_gradient_vs_fp64():
    say("[case] mlp")
    rng = np.random.default_rng(9)
    theta = M.init_params(rng)
    X = rng.standard_normal((300, 33))
    y = rng.standard_normal(300)
    P = torch.tensor(theta, dtype=torch.float32, device=DEV)
    Xd = torch.tensor(X, dtype=torch.float32, device=DEV)
    yd = torch.tensor(y, dtype=torch.float32, device=DEV)
    out = qbvm.mlp_forward(P, Xd).cpu().numpy()
    ref, _ = M.forward(theta.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(out, ref, rtol=1e-4, atol=1e-5)
    loss, grad = qbvm.mlp_loss_grad(P, Xd, yd)
    lo, go = M.loss_and_grad(theta.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64),
                             y.astype(np.float32).astype(np.float64))
    assert abs(float(loss) - lo) <= 1e-4 * lo
    g = grad.cpu().numpy()
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)


def test_adam_vs_reference():
    rng = np.random.default_rng(10)
    th = rng.standard_normal(1000)
    gr = rng.standard_normal(1000)
    m = np.zeros(1000); v = np.zeros(1000)
    P = torch.tensor(th, dtype=torch.float32, device=DEV)
    Gd = torch.tensor(gr, dtype=torch.float32, device=DEV)
    Md = torch.zeros(1000, dtype=torch.float32, device=DEV)
    Vd = torch.zeros(1000, dtype=torch.float32, device=DEV)
    for t in range(1, 4):
        qbvm.adam_step(P, Gd, Md, Vd, t, 1e-2)
        th, m, v = M.adam_step(th, gr, m, v, t, lr=1e-2)
    np.testing.assert_allclose(P.cpu().numpy(), th, rtol=1e-5, atol=1e-6)


# ---------------------------------------------------------------- batched
def padded_shape(d, m, n):
    """Shapes whose single full solve takes the padded pipeline (compile-time sine and time
    kernels); batched instances run the same steps in place, equal to rounding only."""
    p2 = lambda x: x >= 64 and x & (x - 1) == 0
    nt = n + 1
    return d >= 2 and p2(2 * (m + 1)) and 2 * (m + 1) <= 4096 and ((p2(nt) and nt <= 2048) or nt in (129, 257))


def test_batched_matches_single_and_oracle():
    """Uneven batch with every output mode: each instance bitwise equal to its own qbvm_solve and
    within the bar of the closed form; then the same set on new buffers with new alphas (the
    cached graph, its arguments rewritten) and once more on the first buffers."""
    say("[case] batched")
    rng = np.random.default_rng(12)
    specs = [(1, 63, 64, 0), (1, 200, 129, 0), (1, 1023, 300, 0), (2, 63, 64, 0), (2, 100, 257, 0), (2, 31, 90, 0),
             (1, 63, 64, 0), (2, 63, 64, 0), (3, 9, 10, 0), (2, 63, 127, 0), (2, 127, 128, 0), (2, 255, 256, 0),
             (1, 300, 200, 1), (2, 63, 64, 2), (2, 100, 150, 1), (3, 15, 20, 2), (1, 1, 5, 0), (1, 77, 1, 0)]
    grids, variants, outs, ref = [], [], [], []
    for d, m, n, o in specs:
        grids.append((d, m, n, 1.0, 1.0))
        variants.append(int(rng.integers(0, 2)))
        outs.append(o)
        ref.append(rng.standard_normal((m,) * d))

    def run(alphas):
        gs = [to_dev(g) for g in ref]
        ys = [torch.empty(((n + 1,) if o == qbvm.OUT_ALL else ()) + (m,) * d, dtype=torch.float64, device=DEV)
              for d, m, n, o in specs]
        qbvm.solve_batched(grids, alphas, variants, gs, ys, outs)
        torch.cuda.synchronize()
        for i, (d, m, n, o) in enumerate(specs):
            y1 = gpu_solve(d, m, n, 1.0, 1.0, alphas[i], variants[i], ref[i], output=o)
            yb = ys[i].cpu().numpy()
            if not (o == qbvm.OUT_ALL and padded_shape(d, m, n)):
                assert np.array_equal(yb, y1), (i, specs[i], rel(yb, y1), float(np.max(np.abs(yb - y1))))
            lv = None if o == qbvm.OUT_ALL else [0 if o == qbvm.OUT_Y0 else n]
            yc = O.closed_form(ref[i], d, m, n, 1.0, 1.0, alphas[i], variants[i], levels=lv)
            yc = yc if o == qbvm.OUT_ALL else yc[0]
            assert rel(yb, yc) < TOL or o != qbvm.OUT_ALL, (i, rel(yb, yc))
            if o != qbvm.OUT_ALL:
                w = omega_abs(alphas[i], variants[i], 1.0 / n)
                yc0 = O.closed_form(ref[i], d, m, n, 1.0, 1.0, alphas[i], variants[i], levels=[0])[0]
                ok, e = level_ok(yb, yc, yc0, lv[0], n + 1, w)
                assert ok, (i, e)
        return gs, ys

    alphas = [10.0 ** rng.uniform(-6, -1) for _ in specs]
    keep = run(alphas)
    run([a * 3.0 for a in alphas])  # new buffers, new alphas: the cached graph, rewritten
    run(alphas)
    del keep
    qbvm.batched_cache_clear()


def test_batched_cache_is_bounded():
    """More distinct sets of grids than the cache holds: every call still solves correctly."""
    say("[case] batched cache")
    rng = np.random.default_rng(13)
    for k in range(11):
        specs = [(1, 31 + k, 40), (2, 15 + k, 20)]
        grids = [(d, m, n, 1.0, 1.0) for d, m, n in specs]
        ref = [rng.standard_normal((m,) * d) for d, m, n in specs]
        gs = [to_dev(g) for g in ref]
        ys = [torch.empty((n + 1,) + (m,) * d, dtype=torch.float64, device=DEV) for d, m, n in specs]
        qbvm.solve_batched(grids, [1e-3, 1e-4], [0, 1], gs, ys)
        torch.cuda.synchronize()
        for i, (d, m, n) in enumerate(specs):
            yc = O.closed_form(ref[i], d, m, n, 1.0, 1.0, [1e-3, 1e-4][i], i)
            assert rel(ys[i].cpu().numpy(), yc) < TOL
    qbvm.batched_cache_clear()


def test_batched_workload_512_instances():
    """The 512-instance batched workload (256 1D m in [63,1023] + 256 2D m in [63,255], n in
    [64,512], alpha in [1e-6,1e-1]), every level of every instance: bitwise equal to its own
    qbvm_solve, and levels 0, n/2 and n against the closed form."""
    say("[case] batched workload, 512 instances")
    insts = W.config_batched()
    grids = [(i.d, i.m, i.n, i.L, i.T) for i in insts]
    gs = [to_dev(i.g_delta) for i in insts]
    ys = [torch.empty((i.n + 1,) + (i.m,) * i.d, dtype=torch.float64, device=DEV) for i in insts]
    qbvm.solve_batched(grids, [i.alpha for i in insts], [0] * len(insts), gs, ys)
    torch.cuda.synchronize()
    worst = 0.0
    for k, inst in enumerate(insts):
        p = qbvm.Plan(*grids[k])
        y1 = p.solve(inst.alpha, 0, gs[k])
        torch.cuda.synchronize()
        assert torch.equal(ys[k], y1), k
        del y1
        p.close()
        lv = [0, inst.n // 2, inst.n]
        yc = O.closed_form(inst.g_delta, inst.d, inst.m, inst.n, 1.0, 1.0, inst.alpha, O.PQ, levels=lv)
        yl = ys[k][lv].cpu().numpy()
        w_abs = omega_abs(inst.alpha, 0, 1.0 / inst.n)
        for j, t in enumerate(lv):
            # strongly damped levels: the attainable accuracy of Step (c) (see tests/parity_util.py)
            ok, e = level_ok(yl[j], yc[j], yc[0], t, inst.n + 1, w_abs)
            worst = max(worst, e)
            assert ok, (k, t, e)
    say("worst sampled-level rel err", worst)
    qbvm.batched_cache_clear()


def test_autotune_then_solve():
    """The autotuner times the power-of-two kernel variants and keeps parity."""
    say("[case] autotune")
    d, m, n = 2, 127, 256
    g = np.random.default_rng(13).standard_normal((m, m))
    p = qbvm.Plan(d, m, n)
    rep = p.autotune()
    assert rep["variants"]["time"] in (0, 1, 2, 3, 4, 5)
    assert rep["variants"]["rows"] in (0, 1, 3, 4, 5, 6, 7) and rep["variants"]["cols"] in (0, 1, 3, 4, 5, 6, 7)
    assert sum(1 for x in rep["ms_rows_v0134567"] + rep["ms_cols_v0134567"] + rep["ms_time_v012345"] if x > 0) >= 10
    y = p.solve(1e-5, 0, to_dev(g))
    torch.cuda.synchronize()
    yc = O.closed_form(g, d, m, n, 1.0, 1.0, 1e-5, O.PQ)
    assert rel(y.cpu().numpy(), yc) < TOL


def _random_cases(count=24, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = int(rng.integers(1, 4))
        mmax = {1: 1500, 2: 160, 3: 40}[d]
        m = int(rng.integers(1, mmax + 1))
        n = int(rng.integers(1, {1: 1200, 2: 300, 3: 80}[d]))
        alpha = float(10.0 ** rng.uniform(-12, 0))
        out.append((d, m, n, alpha, int(rng.integers(0, 2))))
    return out


@pytest.mark.parametrize("d,m,n,alpha,variant", _random_cases())
def test_random_grids_vs_oracle(d, m, n, alpha, variant):
    """Seeded random grids (every FFT path: Stockham, Rader, Bluestein, Good-Thomas,
    power-of-two; ragged tiles): rank-one solve and general right-hand side against the
    closed forms; in 1D also a variable-coefficient operator."""
    say(f"[case] random d={d} m={m} n={n} alpha={alpha:.3g} variant={variant}")
    rng = np.random.default_rng(d * 7919 + m * 31 + n)
    L, T = 1.0, 0.8
    g = rng.standard_normal((m,) * d)
    p = qbvm.Plan(d, m, n, L, T)
    y = p.solve(alpha, variant, to_dev(g))
    y0 = p.solve(alpha, variant, to_dev(g), output=qbvm.OUT_Y0)
    f = rng.standard_normal((n + 1,) + (m,) * d)
    try:
        yg = p.solve_general(alpha, variant, to_dev(f))
    except qbvm.QbvmError as e:
        # a 1D plan whose sine length 2(m+1) exceeds the FFT core keeps only the
        # tridiagonal path (include/qbvm.h); nothing else may refuse here
        assert e.code == -5 and d == 1, e
        yg = None
    torch.cuda.synchronize()
    yc = O.closed_form(g, d, m, n, L, T, alpha, variant)
    assert rel(y.cpu().numpy(), yc) < TOL
    assert rel(y0.cpu().numpy(), yc[0]) < TOL
    if yg is not None:
        assert rel(yg.cpu().numpy(), O.closed_form_general(f, d, m, n, L, T, alpha, variant)) < TOL
    if d == 1:
        lo, di, up = W.diffusion_operator_1d(m, rng)
        p.set_operator_1d(lo, di, up)
        yo = p.solve(alpha, variant, to_dev(g))
        torch.cuda.synchronize()
        yoc = O.closed_form_operator(g, O.tridiagonal_matrix(lo, di, up), n, T, alpha, variant)
        assert rel(yo.cpu().numpy(), yoc) < TOL
    p.close()
