"""Comparison rule shared by the parity tests.

Levels are compared in the relative 2-norm with the bar 1e-8.  Step (c) forms
level l as gamma_l^{-1}/N_t times a DFT of the N_t shifted solutions, whose
rounding error is about eps * |omega|^{-l/N_t} times the size of that DFT's input
(which is of the order of y^0).  For a level many orders of magnitude smaller
than y^0 (strongly damped data, large alpha) the attainable relative accuracy is
therefore limited; the check then also accepts an absolute error below
FLOOR * eps * |omega|^{-l/N_t} * ||y^0||.
"""
import math

import numpy as np

BAR = 1e-8
FLOOR = 1e3  # generous multiple of the rounding estimate


def omega_abs(alpha: float, variant: int, tau: float) -> float:
    return 1.0 / alpha if variant == 0 else tau / alpha


def level_ok(y_l, yc_l, yc_0, l: int, Nt: int, w_abs: float):
    err = float(np.linalg.norm(np.ravel(y_l - yc_l)))
    ref = float(np.linalg.norm(np.ravel(yc_l)))
    floor = FLOOR * np.finfo(float).eps * math.exp(-l / Nt * math.log(w_abs)) * float(
        np.linalg.norm(np.ravel(yc_0)))
    return err <= BAR * ref or err <= floor, err / max(ref, 1e-300)
