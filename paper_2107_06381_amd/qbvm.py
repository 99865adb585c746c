"""Thin Python binding of libqbvm.so (the C ABI declared in include/qbvm.h).

Argument marshalling only: tensors are checked for device, dtype, contiguity and
size, then their device pointers and the current HIP stream are passed to the
library, where every step of the solve runs.  PyTorch supplies device memory and
streams.  There is no CPU fallback: if the library cannot be loaded, every call
raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqbvm.so")

QBVM_PQ, QBVM_PM = 0, 1
OUT_ALL, OUT_Y0, OUT_YN = 0, 1, 2
MLP_PARAMS = 6401
MODEL_FLOATS = 6469
NFEAT = 33

ERR_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOROOT", -5: "EUNSUPPORTED",
             -6: "ENOMODEL", -7: "ENOCONV"}

# every symbol include/qbvm.h declares
EXPORTS = [
    "qbvm_plan", "qbvm_plan_destroy", "qbvm_plan_set_stream", "qbvm_plan_workspace_bytes",
    "qbvm_solve", "qbvm_solve_general", "qbvm_solve_batched", "qbvm_batched_cache_clear", "qbvm_discrepancy",
    "qbvm_choose_alpha", "qbvm_choose_alpha_each", "qbvm_bisect_batched", "qbvm_features", "qbvm_set_alpha_model",
    "qbvm_mlp_forward", "qbvm_mlp_loss_grad", "qbvm_mlp_loss_grad_noalloc", "qbvm_adam_step", "qbvm_strerror",
    "qbvm_last_error", "qbvm_version", "qbvm_profile_enable", "qbvm_profile_reset",
    "qbvm_profile_count", "qbvm_profile_get", "qbvm_plan_autotune", "qbvm_plan_get_variants",
    "qbvm_plan_set_variants", "qbvm_plan_set_operator_1d", "qbvm_plan_set_plane", "qbvm_plan_get_plane",
    "qbvm_plan_set_operator_2d", "qbvm_plan_set_operator_3d", "qbvm_plan_operator_stats",
]


class QbvmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qbvm error {code} ({ERR_NAMES.get(code, '?')}): {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("m", ctypes.c_int), ("n", ctypes.c_int),
                ("L", ctypes.c_double), ("T", ctypes.c_double)]


class AlphaOpts(ctypes.Structure):
    _fields_ = [("tau_dp", ctypes.c_double), ("log10_lo", ctypes.c_double),
                ("log10_hi", ctypes.c_double), ("steps", ctypes.c_int),
                ("use_learned", ctypes.c_int), ("win_lo", ctypes.c_double),
                ("win_hi", ctypes.c_double)]


class AlphaInfo(ctypes.Structure):
    _fields_ = [("discrepancy", ctypes.c_double), ("alpha_learned", ctypes.c_double),
                ("iterations", ctypes.c_int), ("used_fallback", ctypes.c_int),
                ("bracket_hit", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libqbvm.so (built by paper_2107_06381_amd.build); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2107_06381_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has loaded, so both share
    # one runtime (a second copy of the runtime in the process would not see the device)
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, i, d, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    sig = {
        "qbvm_plan": (i, [ctypes.POINTER(vp), ctypes.POINTER(Grid), vp]),
        "qbvm_plan_destroy": (None, [vp]),
        "qbvm_plan_set_stream": (i, [vp, vp]),
        "qbvm_plan_workspace_bytes": (ll, [vp]),
        "qbvm_solve": (i, [vp, d, i, vp, vp, i]),
        "qbvm_solve_general": (i, [vp, d, i, vp, vp]),
        "qbvm_solve_batched": (i, [i, ctypes.POINTER(Grid), ctypes.POINTER(d), ctypes.POINTER(i),
                                   ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i), vp]),
        "qbvm_batched_cache_clear": (None, []),
        "qbvm_discrepancy": (i, [vp, d, i, vp, ctypes.POINTER(d)]),
        "qbvm_choose_alpha": (i, [vp, i, vp, d, ctypes.POINTER(AlphaOpts), ctypes.POINTER(d),
                                  ctypes.POINTER(AlphaInfo)]),
        "qbvm_choose_alpha_each": (i, [vp, i, i, vp, ctypes.POINTER(d), ctypes.POINTER(AlphaOpts),
                                       ctypes.POINTER(d), ctypes.POINTER(AlphaInfo), ctypes.POINTER(d)]),
        "qbvm_bisect_batched": (i, [vp, i, i, vp, vp, ctypes.POINTER(AlphaOpts), vp, vp]),
        "qbvm_features": (i, [vp, i, vp, vp, vp]),
        "qbvm_set_alpha_model": (i, [vp, ctypes.POINTER(ctypes.c_float)]),
        "qbvm_mlp_forward": (i, [vp, i, vp, vp, vp]),
        "qbvm_mlp_loss_grad": (i, [vp, i, vp, vp, vp, vp, vp]),
        "qbvm_mlp_loss_grad_noalloc": (i, [vp, i, vp, vp, vp, vp, vp]),
        "qbvm_adam_step": (i, [vp, vp, vp, vp, i, i, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, vp]),
        "qbvm_strerror": (ctypes.c_char_p, [i]),
        "qbvm_last_error": (ctypes.c_char_p, []),
        "qbvm_version": (i, []),
        "qbvm_plan_autotune": (i, [vp, ctypes.POINTER(d)]),
        "qbvm_plan_get_variants": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i),
                                       ctypes.POINTER(i)]),
        "qbvm_plan_set_variants": (i, [vp, i, i, i, i]),
        "qbvm_plan_set_operator_1d": (i, [vp, vp, vp, vp]),
        "qbvm_plan_set_operator_2d": (i, [vp, vp, vp, d, i]),
        "qbvm_plan_set_operator_3d": (i, [vp, vp, vp, vp, d, i]),
        "qbvm_plan_operator_stats": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(d), ctypes.POINTER(i)]),
        "qbvm_plan_set_plane": (i, [vp, i]),
        "qbvm_plan_get_plane": (i, [vp, ctypes.POINTER(i)]),
        "qbvm_profile_enable": (None, [i]),
        "qbvm_profile_reset": (None, []),
        "qbvm_profile_count": (i, []),
        "qbvm_profile_get": (i, [i, ctypes.c_char_p, i, ctypes.POINTER(ll), ctypes.POINTER(d),
                                 ctypes.POINTER(d), ctypes.POINTER(d)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        L = load()
        raise QbvmError(rc, f"{L.qbvm_strerror(rc).decode()}: {L.qbvm_last_error().decode()}")


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_tensor(t, numel: int, dtype, name: str):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def default_alpha_opts(use_learned: bool = False) -> AlphaOpts:
    return AlphaOpts(1.1, -20.0, 0.0, 30, 1 if use_learned else 0, 1.05, 1.15)


class Plan:
    """A grid-bound solver plan (qbvm_plan): d, m, n, L, T and a HIP stream."""

    def __init__(self, d: int, m: int, n: int, L: float = 1.0, T: float = 1.0, stream=None):
        import torch
        self.L_ = load()
        self.d, self.m, self.n, self.Lx, self.T = int(d), int(m), int(n), float(L), float(T)
        self.nmodes = self.m ** self.d
        self.device = torch.cuda.current_device()
        self._stream = stream
        self._h = ctypes.c_void_p()
        g = Grid(self.d, self.m, self.n, self.Lx, self.T)
        _check(self.L_.qbvm_plan(ctypes.byref(self._h), ctypes.byref(g), ctypes.c_void_p(_stream(stream))))

    def close(self):
        if self._h:
            self.L_.qbvm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self) -> int:
        return int(self.L_.qbvm_plan_workspace_bytes(self._h))

    def autotune(self) -> dict:
        """Time the kernel variants on this plan's shape and keep the fastest."""
        ms = (ctypes.c_double * 30)()
        _check(self.L_.qbvm_plan_autotune(self._h, ms))
        v = [round(x, 5) for x in ms]
        return {"ms_rows_v0134567": v[0:7], "ms_cols_v0134567": v[7:14], "ms_time_v012345": v[14:20],
                "ms_general_v012345": v[20:26], "ms_separate_x2_x1": v[26], "ms_plane_v012": v[27:30],
                "variants": self.variants(), "plane_variant": self.plane_variant()}

    def variants(self):
        r, c, t, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self.L_.qbvm_plan_get_variants(self._h, ctypes.byref(r), ctypes.byref(c), ctypes.byref(t),
                                              ctypes.byref(g)))
        return {"rows": r.value, "cols": c.value, "time": t.value, "general": g.value}

    def set_operator_1d(self, lower=None, diag=None, upper=None):
        """Tridiagonal spatial operator in place of -Lap_h (1D); diag=None restores it."""
        import numpy as np
        if diag is None:
            _check(self.L_.qbvm_plan_set_operator_1d(self._h, None, None, None))
            return
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (lower, diag, upper)]
        if arrs[1].shape != (self.m,) or arrs[0].shape != (self.m - 1,) or arrs[2].shape != (self.m - 1,):
            raise ValueError("operator diagonals must have m-1, m, m-1 entries")
        ptr = [a.ctypes.data if a.size else None for a in arrs]
        _check(self.L_.qbvm_plan_set_operator_1d(self._h, *ptr))

    def set_operator_2d(self, kx=None, ky=None, tol: float = 1e-12, max_iter: int = 200):
        """-div(kappa grad u) in place of -Lap_h (2D), kappa at the cell faces: kx (m, m+1),
        ky (m+1, m); kx=None restores -Lap_h (qbvm_plan_set_operator_2d)."""
        import numpy as np
        if kx is None:
            _check(self.L_.qbvm_plan_set_operator_2d(self._h, None, None, 0.0, 0))
            return
        kx = np.ascontiguousarray(kx, dtype=np.float64)
        ky = np.ascontiguousarray(ky, dtype=np.float64)
        if kx.shape != (self.m, self.m + 1) or ky.shape != (self.m + 1, self.m):
            raise ValueError("kx must be (m, m+1) and ky (m+1, m)")
        _check(self.L_.qbvm_plan_set_operator_2d(self._h, kx.ctypes.data, ky.ctypes.data, float(tol),
                                                 int(max_iter)))

    def set_operator_3d(self, kx=None, ky=None, kz=None, tol: float = 1e-12, max_iter: int = 200):
        """-div(kappa grad u) in place of -Lap_h (3D), kappa at the cell faces: kx (m, m, m+1),
        ky (m, m+1, m), kz (m+1, m, m); kx=None restores -Lap_h (qbvm_plan_set_operator_3d)."""
        import numpy as np
        if kx is None:
            _check(self.L_.qbvm_plan_set_operator_3d(self._h, None, None, None, 0.0, 0))
            return
        m = self.m
        arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (kx, ky, kz)]
        if [a.shape for a in arrs] != [(m, m, m + 1), (m, m + 1, m), (m + 1, m, m)]:
            raise ValueError("kx, ky, kz must be (m, m, m+1), (m, m+1, m), (m+1, m, m)")
        _check(self.L_.qbvm_plan_set_operator_3d(self._h, *(a.ctypes.data for a in arrs), float(tol),
                                                 int(max_iter)))

    def operator_stats(self) -> dict:
        """Iterations, largest relative residual and breakdowns of the last 2D-operator solve."""
        it, br = ctypes.c_int(), ctypes.c_int()
        rr = ctypes.c_double()
        _check(self.L_.qbvm_plan_operator_stats(self._h, ctypes.byref(it), ctypes.byref(rr), ctypes.byref(br)))
        return {"iterations": it.value, "max_rel_residual": rr.value, "breakdowns": br.value}

    def set_variants(self, rows: int = -1, cols: int = -1, time: int = -1, general: int = -1):
        """Select kernel variants by hand (-1 keeps the current one)."""
        _check(self.L_.qbvm_plan_set_variants(self._h, int(rows), int(cols), int(time), int(general)))

    def set_plane(self, on: bool, variant: int = 0):
        """qbvm_plan_set_plane: the x_2/x_1 plane pass (this variant) on, or off."""
        _check(self.L_.qbvm_plan_set_plane(self._h, int(variant) if on else -1))

    def plane_variant(self) -> int:
        """Plane-pass variant qbvm_solve uses, -1 for the separate passes."""
        v = ctypes.c_int()
        _check(self.L_.qbvm_plan_get_plane(self._h, ctypes.byref(v)))
        return v.value

    def uses_plane(self) -> bool:
        return self.plane_variant() >= 0

    def out_shape(self, output: int):
        sp = (self.m,) * self.d
        return ((self.n + 1,) + sp) if output == OUT_ALL else sp

    def solve(self, alpha: float, variant: int, g_delta, y=None, output: int = OUT_ALL):
        import torch
        if y is None:
            y = torch.empty(self.out_shape(output), dtype=torch.float64, device=g_delta.device)
        gp = _dev_tensor(g_delta, self.nmodes, torch.float64, "g_delta")
        nout = self.nmodes * ((self.n + 1) if output == OUT_ALL else 1)
        yp = _dev_tensor(y, nout, torch.float64, "y")
        _check(self.L_.qbvm_solve(self._h, float(alpha), int(variant), gp, yp, int(output)))
        return y

    def solve_general(self, alpha: float, variant: int, f, y=None):
        """All-at-once system with right-hand side f ((n+1, m, ..) levels) -> y (may be f)."""
        import torch
        if y is None:
            y = torch.empty(self.out_shape(OUT_ALL), dtype=torch.float64, device=f.device)
        n = self.nmodes * (self.n + 1)
        fp = _dev_tensor(f, n, torch.float64, "f")
        yp = _dev_tensor(y, n, torch.float64, "y")
        _check(self.L_.qbvm_solve_general(self._h, float(alpha), int(variant), fp, yp))
        return y

    def discrepancy(self, alpha: float, variant: int, g_delta) -> float:
        import torch
        gp = _dev_tensor(g_delta, self.nmodes, torch.float64, "g_delta")
        D = ctypes.c_double()
        _check(self.L_.qbvm_discrepancy(self._h, float(alpha), int(variant), gp, ctypes.byref(D)))
        return D.value

    def choose_alpha(self, variant: int, g_delta, delta: float, opts: Optional[AlphaOpts] = None,
                     raise_on_noroot: bool = False):
        import torch
        opts = opts or default_alpha_opts()
        gp = _dev_tensor(g_delta, self.nmodes, torch.float64, "g_delta")
        a = ctypes.c_double()
        info = AlphaInfo()
        rc = self.L_.qbvm_choose_alpha(self._h, int(variant), gp, float(delta), ctypes.byref(opts),
                                       ctypes.byref(a), ctypes.byref(info))
        if rc == -4 and not raise_on_noroot:
            return a.value, info
        _check(rc)
        return a.value, info

    def choose_alpha_each(self, variant: int, g_deltas, deltas, opts: Optional[AlphaOpts] = None):
        """qbvm_choose_alpha_each: one call per instance, timed in the library.  g_deltas: GPU
        tensor (count, m, ..); deltas: host sequence.  Returns (alphas, infos, seconds) as numpy
        arrays (infos: structured fields alpha_learned, iterations, used_fallback, bracket_hit)."""
        import numpy as np
        import torch
        opts = opts or default_alpha_opts()
        dl = np.ascontiguousarray(np.asarray(deltas, dtype=np.float64).ravel())
        count = int(dl.size)
        gp = _dev_tensor(g_deltas, count * self.nmodes, torch.float64, "g_deltas")
        alphas = np.empty(count)
        secs = np.empty(count)
        infos = (AlphaInfo * max(1, count))()
        dptr = ctypes.POINTER(ctypes.c_double)
        _check(self.L_.qbvm_choose_alpha_each(self._h, int(variant), count, gp, dl.ctypes.data_as(dptr),
                                              ctypes.byref(opts), alphas.ctypes.data_as(dptr), infos,
                                              secs.ctypes.data_as(dptr)))
        rec = np.array([(x.discrepancy, x.alpha_learned, x.iterations, x.used_fallback, x.bracket_hit)
                        for x in infos[:count]],
                       dtype=[("discrepancy", "f8"), ("alpha_learned", "f8"), ("iterations", "i4"),
                              ("used_fallback", "i4"), ("bracket_hit", "i4")])
        return alphas, rec, secs

    def bisect_batched(self, variant: int, g_deltas, deltas, opts: Optional[AlphaOpts] = None):
        import torch
        opts = opts or default_alpha_opts()
        count = int(deltas.numel())
        gp = _dev_tensor(g_deltas, count * self.nmodes, torch.float64, "g_deltas")
        dp = _dev_tensor(deltas, count, torch.float64, "deltas")
        alphas = torch.empty(count, dtype=torch.float64, device=deltas.device)
        hits = torch.empty(count, dtype=torch.int32, device=deltas.device)
        _check(self.L_.qbvm_bisect_batched(self._h, int(variant), count, gp, dp, ctypes.byref(opts),
                                           ctypes.c_void_p(alphas.data_ptr()),
                                           ctypes.c_void_p(hits.data_ptr())))
        return alphas, hits

    def features(self, g_deltas, deltas):
        import torch
        count = int(deltas.numel())
        gp = _dev_tensor(g_deltas, count * self.nmodes, torch.float64, "g_deltas")
        dp = _dev_tensor(deltas, count, torch.float64, "deltas")
        f = torch.empty((count, NFEAT), dtype=torch.float32, device=deltas.device)
        _check(self.L_.qbvm_features(self._h, count, gp, dp, ctypes.c_void_p(f.data_ptr())))
        return f

    def set_alpha_model(self, model):
        """model: host float32 array-like of MODEL_FLOATS values."""
        import numpy as np
        arr = np.ascontiguousarray(np.asarray(model, dtype=np.float32).ravel())
        if arr.size != MODEL_FLOATS:
            raise ValueError(f"model must have {MODEL_FLOATS} floats")
        _check(self.L_.qbvm_set_alpha_model(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))


def solve_batched(grids: Sequence[tuple], alphas: Sequence[float], variants: Sequence[int],
                  g_deltas: Sequence, ys: Sequence, outputs: Optional[Sequence[int]] = None, stream=None):
    """qbvm_solve_batched: grids are (d, m, n, L, T) tuples; tensors on the GPU."""
    import torch
    L_ = load()
    count = len(grids)
    outputs = outputs if outputs is not None else [OUT_ALL] * count
    G = (Grid * count)(*[Grid(int(g[0]), int(g[1]), int(g[2]), float(g[3]), float(g[4])) for g in grids])
    A = (ctypes.c_double * count)(*[float(a) for a in alphas])
    V = (ctypes.c_int * count)(*[int(v) for v in variants])
    O = (ctypes.c_int * count)(*[int(o) for o in outputs])
    gp, yp = [], []
    for i, (g, (d, m, n, _, _)) in enumerate(zip(g_deltas, grids)):
        nm = int(m) ** int(d)
        gp.append(_dev_tensor(g, nm, torch.float64, f"g_deltas[{i}]").value)
        nout = nm * ((int(n) + 1) if outputs[i] == OUT_ALL else 1)
        yp.append(_dev_tensor(ys[i], nout, torch.float64, f"ys[{i}]").value)
    GP = (ctypes.c_void_p * count)(*gp)
    YP = (ctypes.c_void_p * count)(*yp)
    _check(L_.qbvm_solve_batched(count, G, A, V, GP, YP, O, ctypes.c_void_p(_stream(stream))))


def batched_cache_clear():
    load().qbvm_batched_cache_clear()


def mlp_forward(params, X, out=None, stream=None):
    import torch
    B = X.shape[0]
    out = out if out is not None else torch.empty(B, dtype=torch.float32, device=X.device)
    _check(load().qbvm_mlp_forward(_dev_tensor(params, MLP_PARAMS, torch.float32, "params"), B,
                                   _dev_tensor(X, B * NFEAT, torch.float32, "X"),
                                   _dev_tensor(out, B, torch.float32, "out"),
                                   ctypes.c_void_p(_stream(stream))))
    return out


def mlp_loss_grad(params, X, y, grad=None, loss=None, stream=None):
    import torch
    B = X.shape[0]
    grad = grad if grad is not None else torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
    loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=X.device)
    _check(load().qbvm_mlp_loss_grad(_dev_tensor(params, MLP_PARAMS, torch.float32, "params"), B,
                                     _dev_tensor(X, B * NFEAT, torch.float32, "X"),
                                     _dev_tensor(y, B, torch.float32, "y"),
                                     _dev_tensor(grad, MLP_PARAMS, torch.float32, "grad"),
                                     _dev_tensor(loss, 1, torch.float32, "loss"),
                                     ctypes.c_void_p(_stream(stream))))
    return loss, grad


NOALLOC_MAX_BATCH = 16384


def mlp_loss_grad_noalloc(params, X, y, grad, loss, stream=None):
    """qbvm_mlp_loss_grad_noalloc: the caller passes grad and loss; the library allocates nothing."""
    import torch
    B = X.shape[0]
    _check(load().qbvm_mlp_loss_grad_noalloc(_dev_tensor(params, MLP_PARAMS, torch.float32, "params"), B,
                                             _dev_tensor(X, B * NFEAT, torch.float32, "X"),
                                             _dev_tensor(y, B, torch.float32, "y"),
                                             _dev_tensor(grad, MLP_PARAMS, torch.float32, "grad"),
                                             _dev_tensor(loss, 1, torch.float32, "loss"),
                                             ctypes.c_void_p(_stream(stream))))
    return loss, grad


def adam_step(params, grad, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8, stream=None):
    import torch
    n = params.numel()
    _check(load().qbvm_adam_step(_dev_tensor(params, n, torch.float32, "params"),
                                 _dev_tensor(grad, n, torch.float32, "grad"),
                                 _dev_tensor(m, n, torch.float32, "m"),
                                 _dev_tensor(v, n, torch.float32, "v"), n, int(step), float(lr),
                                 float(b1), float(b2), float(eps), ctypes.c_void_p(_stream(stream))))


def profile_enable(on: bool = True):
    load().qbvm_profile_enable(1 if on else 0)


def profile_reset():
    load().qbvm_profile_reset()


def profile_report() -> dict:
    """{kernel kind: {launches, total_ms, bytes, flops}} folded from the recorded events."""
    L_ = load()
    out = {}
    for i in range(L_.qbvm_profile_count()):
        name = ctypes.create_string_buffer(64)
        n = ctypes.c_longlong()
        ms, by, fl = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(L_.qbvm_profile_get(i, name, 64, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                   ctypes.byref(fl)))
        out[name.value.decode()] = {"launches": n.value, "total_ms": ms.value, "bytes": by.value,
                                    "flops": fl.value}
    return out
