"""Seeded synthetic workloads for the backward heat conduction problem.

This module only *produces inputs*: an initial datum z0 on the interior grid, the
noise-free final state g that the forward heat equation carries it to, and the
noisy measurement g_delta with its noise level delta.  It contains none of the
regularised (quasi-boundary value) solve; the CPU oracle and the GPU library
both consume what it returns and neither is imported here.

Problem statement (Section 1, eq. "state"): z_t - Lap z = 0 on Omega=(0,L)^d with
homogeneous Dirichlet data; the final state g = z(.,T) is observed with noise,
||g - g_delta|| <= delta.

Discretisation used for g (Section 2): uniform mesh with m interior points per
dimension, h = L/(m+1), backward Euler with tau = T/n.  The discrete forward map
is g = (I - tau Lap_h)^{-n} z0.  Its evaluation below uses the discrete sine
eigenvectors of the Dirichlet stencil (a textbook fact about the forward heat
equation, not part of the regularised solve); a test checks it against a literal
step-by-step backward-Euler march.

Norm convention: the paper's "discrete L2(Omega) norm" (Section 5) is read as
||v||_h = h^{d/2} ||v||_2; delta is reported in that norm.  Noise is relative
Gaussian: g_delta = g + eps ||g|| eta/||eta||, so delta = eps ||g||_h exactly.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.fft as _sfft

__all__ = [
    "Instance", "nodes", "forward_final_state_modes", "forward_final_state_dense",
    "add_relative_noise", "sine_mode_instance", "config_1d", "config_2d", "config_3d",
    "config_batched", "config_learned", "weighted_norm",
]


@dataclasses.dataclass
class Instance:
    d: int
    m: int
    n: int
    L: float
    T: float
    alpha: float
    variant: int          # 0 = PinT-QBVM, 1 = PinT-MQBVM
    g_delta: np.ndarray   # shape (m,)*d, C order, last axis = x_1 (fastest)
    delta: float          # noise level in the h-weighted norm
    z0: np.ndarray        # exact initial datum on the interior nodes
    g: np.ndarray         # noise-free final state
    eps: float = 0.0

    @property
    def unknowns_nmd(self) -> int:
        return self.n * self.m ** self.d

    @property
    def unknowns_true(self) -> int:
        return (self.n + 1) * self.m ** self.d


def nodes(m: int, L: float) -> np.ndarray:
    """Interior nodes x_i = i h, i = 1..m, h = L/(m+1)."""
    h = L / (m + 1)
    return h * np.arange(1, m + 1, dtype=np.float64)


def weighted_norm(v: np.ndarray, h: float, d: int) -> float:
    return float(h ** (d / 2.0) * np.linalg.norm(np.ravel(v)))


def _stencil_eig_1d(k: np.ndarray, m: int, L: float) -> np.ndarray:
    # eigenvalue of the 3-point Dirichlet stencil -(u_{i-1}-2u_i+u_{i+1})/h^2 on sin(k pi x/L)
    h = L / (m + 1)
    return (4.0 / (h * h)) * np.sin(k * np.pi / (2.0 * (m + 1))) ** 2


def forward_final_state_modes(modes: np.ndarray, coef: np.ndarray, m: int, n: int,
                              L: float, T: float) -> tuple[np.ndarray, np.ndarray]:
    """z0 = sum_c coef_c prod_i sin(k_{c,i} pi x_i / L) and g = (I - tau Lap_h)^{-n} z0.

    modes: (C, d) integer wave numbers in 1..m; coef: (C,).
    Returns (z0, g) with shape (m,)*d, axis order (x_d, ..., x_1).
    """
    modes = np.asarray(modes, dtype=np.int64)
    C, d = modes.shape
    tau = T / n
    x = nodes(m, L)
    lam = np.zeros(C)
    for i in range(d):
        lam += _stencil_eig_1d(modes[:, i].astype(np.float64), m, L)
    decay = (1.0 / (1.0 + tau * lam)) ** n
    # separable evaluation: for each mode, outer product of 1D sines.
    # axis order in the array is (x_d, ..., x_1): modes[:, 0] is the x_1 wave number.
    sines = [np.sin(np.outer(modes[:, i], x) * np.pi / L) for i in range(d)]  # (C, m)
    if d == 1:
        z0 = coef @ sines[0]
        g = (coef * decay) @ sines[0]
    elif d == 2:
        z0 = np.einsum("c,ci,cj->ji", coef, sines[0], sines[1])
        g = np.einsum("c,ci,cj->ji", coef * decay, sines[0], sines[1])
    elif d == 3:
        z0 = np.einsum("c,ci,cj,ck->kji", coef, sines[0], sines[1], sines[2])
        g = np.einsum("c,ci,cj,ck->kji", coef * decay, sines[0], sines[1], sines[2])
    else:
        raise ValueError("d must be 1, 2 or 3")
    return np.ascontiguousarray(z0), np.ascontiguousarray(g)


def forward_final_state_dense(z0: np.ndarray, n: int, L: float, T: float) -> np.ndarray:
    """g = (I - tau Lap_h)^{-n} z0 for an arbitrary grid function z0 (any d).

    Uses the orthonormal type-I discrete sine transform (its basis vectors are the
    eigenvectors of the Dirichlet stencil along every axis).
    """
    d = z0.ndim
    m = z0.shape[0]
    tau = T / n
    k = np.arange(1, m + 1, dtype=np.float64)
    lam1 = _stencil_eig_1d(k, m, L)
    lam = np.zeros((m,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = m
        lam = lam + lam1.reshape(shape)
    zh = _sfft.dstn(z0, type=1, norm="ortho")
    gh = zh * (1.0 / (1.0 + tau * lam)) ** n
    return np.ascontiguousarray(_sfft.idstn(gh, type=1, norm="ortho"))


def add_relative_noise(g: np.ndarray, eps: float, rng: np.random.Generator,
                       h: float) -> tuple[np.ndarray, float]:
    """g_delta = g + eps ||g|| eta/||eta||, eta iid N(0,1) in C order; delta = eps ||g||_h."""
    eta = rng.standard_normal(g.shape)
    gn = float(np.linalg.norm(g.ravel()))
    en = float(np.linalg.norm(eta.ravel()))
    g_delta = g + (eps * gn / en) * eta
    delta = eps * gn * h ** (g.ndim / 2.0)
    return np.ascontiguousarray(g_delta), float(delta)


def _lowest_modes(d: int, m: int) -> np.ndarray:
    """The 64 lowest wave numbers: 8^d... read as 8x8 in 2D, k=1..64 in 1D, 4x4x4 in 3D."""
    if d == 1:
        kk = np.arange(1, min(64, m) + 1)
        return kk[:, None]
    if d == 2:
        r = np.arange(1, min(8, m) + 1)
        k2, k1 = np.meshgrid(r, r, indexing="ij")
        return np.stack([k1.ravel(), k2.ravel()], axis=1)
    r = np.arange(1, min(4, m) + 1)
    k3, k2, k1 = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([k1.ravel(), k2.ravel(), k3.ravel()], axis=1)


def sine_mode_instance(d: int, m: int, n: int, T: float, alpha: float, eps: float,
                       rng: np.random.Generator, L: float = 1.0, variant: int = 0) -> Instance:
    """Random sine-mode datum: coefficients N(0,1)/(1+|k|^2) on the lowest modes, then noise."""
    modes = _lowest_modes(d, m)
    ksq = np.sum(modes.astype(np.float64) ** 2, axis=1)
    coef = rng.standard_normal(modes.shape[0]) / (1.0 + ksq)
    z0, g = forward_final_state_modes(modes, coef, m, n, L, T)
    h = L / (m + 1)
    g_delta, delta = add_relative_noise(g, eps, rng, h)
    return Instance(d, m, n, L, T, alpha, variant, g_delta, delta, z0, g, eps)


def diffusion_operator_1d(m: int, rng: np.random.Generator, L: float = 1.0, contrast: float = 4.0,
                          advection: float = 0.0):
    """Input data for a 1D problem with another spatial operator: the three diagonals
    (lower[m-1], diag[m], upper[m-1]) of the matrix A that stands in for -Lap_h.
    A is -(kappa u')' + advection u' with Dirichlet ends on the m interior nodes:
    kappa at the half points x_{i+1/2} is smooth and positive (log kappa a sum of
    random low sine modes, max/min about `contrast`), the diffusion term in
    conservative three-point form, the advection term upwinded (advection >= 0).
    advection = 0 gives a symmetric A."""
    h = L / (m + 1)
    xh = (np.arange(m + 1) + 0.5) * h
    k = np.arange(1, 5)
    logk = (rng.standard_normal(4) / k) @ np.sin(np.outer(k, np.pi * xh / L))
    span = float(np.ptp(logk))
    logk *= (np.log(contrast) / span) if span > 0 else 0.0
    kappa = np.exp(logk - logk.mean())
    diag = (kappa[:-1] + kappa[1:]) / h ** 2 + advection / h
    upper = -kappa[1:-1] / h ** 2
    lower = -kappa[1:-1] / h ** 2 - advection / h
    return np.ascontiguousarray(lower), np.ascontiguousarray(diag), np.ascontiguousarray(upper)


def diffusion_coefficients_2d(m: int, rng: np.random.Generator, L: float = 1.0, contrast: float = 4.0):
    """Input data for a 2D problem with the operator -div(kappa grad u): kappa at the cell
    faces of the m x m interior grid (Dirichlet boundary), as two arrays
      kx[j][i], i = 0..m: kappa at (x_1, x_2) = ((i + 1/2) h, (j + 1) h), the face between
                          x_1 nodes i - 1 and i (shape (m, m + 1));
      ky[j][i], j = 0..m: kappa at ((i + 1) h, (j + 1/2) h), between x_2 nodes j - 1 and j
                          (shape (m + 1, m)).
    kappa is smooth and positive: log kappa is a sum of random low sine modes
    sin(k_1 pi x_1) sin(k_2 pi x_2), k_1, k_2 <= 3, scaled so that max/min of kappa over
    the faces is `contrast`, with geometric mean 1 over the faces."""
    h = L / (m + 1)
    k = np.arange(1, 4)
    c = rng.standard_normal((3, 3)) / np.add.outer(k, k)

    def logk(x1, x2):
        return np.einsum("ab,a...,b...->...", c, np.sin(np.multiply.outer(k, np.pi * x1 / L)),
                         np.sin(np.multiply.outer(k, np.pi * x2 / L)))

    nodes = (np.arange(m) + 1.0) * h
    half = (np.arange(m + 1) + 0.5) * h
    lx = logk(*np.meshgrid(half, nodes, indexing="xy"))   # (m, m+1): rows x_2, columns x_1
    ly = logk(*np.meshgrid(nodes, half, indexing="xy"))   # (m+1, m)
    allv = np.concatenate([lx.ravel(), ly.ravel()])
    span = float(np.ptp(allv))
    scale = (np.log(contrast) / span) if span > 0 else 0.0
    mean = float(allv.mean()) * scale
    kx = np.exp(lx * scale - mean)
    ky = np.exp(ly * scale - mean)
    return np.ascontiguousarray(kx), np.ascontiguousarray(ky)


def diffusion_coefficients_3d(m: int, rng: np.random.Generator, L: float = 1.0, contrast: float = 4.0):
    """3D counterpart of diffusion_coefficients_2d: kappa at the faces of the m^3 interior
    grid, arrays indexed [x_3][x_2][x_1] with the face axis extended by one:
    kx (m, m, m+1) at ((i + 1/2) h, (j + 1) h, (k + 1) h), ky (m, m+1, m), kz (m+1, m, m).
    log kappa is a sum of random sin(k_1 pi x_1) sin(k_2 pi x_2) sin(k_3 pi x_3),
    k_1, k_2, k_3 <= 2, scaled to max/min `contrast` over the faces, geometric mean 1."""
    h = L / (m + 1)
    k = np.arange(1, 3)
    c = rng.standard_normal((2, 2, 2)) / (k[:, None, None] + k[None, :, None] + k[None, None, :])

    def logk(x1, x2, x3):
        s1 = np.sin(np.multiply.outer(k, np.pi * x1 / L))
        s2 = np.sin(np.multiply.outer(k, np.pi * x2 / L))
        s3 = np.sin(np.multiply.outer(k, np.pi * x3 / L))
        return np.einsum("abc,a...,b...,c...->...", c, s1, s2, s3)

    nodes = (np.arange(m) + 1.0) * h
    half = (np.arange(m + 1) + 0.5) * h
    # meshgrid with indexing="ij" over (x_3, x_2, x_1)
    X3, X2, X1 = np.meshgrid(nodes, nodes, half, indexing="ij")
    lx = logk(X1, X2, X3)
    X3, X2, X1 = np.meshgrid(nodes, half, nodes, indexing="ij")
    ly = logk(X1, X2, X3)
    X3, X2, X1 = np.meshgrid(half, nodes, nodes, indexing="ij")
    lz = logk(X1, X2, X3)
    allv = np.concatenate([lx.ravel(), ly.ravel(), lz.ravel()])
    span = float(np.ptp(allv))
    scale = (np.log(contrast) / span) if span > 0 else 0.0
    mean = float(allv.mean()) * scale
    return (np.ascontiguousarray(np.exp(lx * scale - mean)), np.ascontiguousarray(np.exp(ly * scale - mean)),
            np.ascontiguousarray(np.exp(lz * scale - mean)))


def config_1d(seed: int = 0, m: int = 127, n: int = 128, alpha: float = 1e-3,
              eps: float = 0.01) -> Instance:
    """1D, (0,1), z0 = sin(pi x) + 0.5 sin(3 pi x), T=1, 1% relative Gaussian noise."""
    rng = np.random.default_rng(seed)
    modes = np.array([[1], [3]])
    coef = np.array([1.0, 0.5])
    z0, g = forward_final_state_modes(modes, coef, m, n, 1.0, 1.0)
    g_delta, delta = add_relative_noise(g, eps, rng, 1.0 / (m + 1))
    return Instance(1, m, n, 1.0, 1.0, alpha, 0, g_delta, delta, z0, g, eps)


def config_2d(seed: int = 1, m: int = 255, n: int = 256, alpha: float = 1e-4,
              eps: float = 0.005) -> Instance:
    """2D, (0,1)^2, 64 random lowest sine modes, T=1, 0.5% relative Gaussian noise."""
    return sine_mode_instance(2, m, n, 1.0, alpha, eps, np.random.default_rng(seed))


def config_3d(seed: int = 2, m: int = 127, n: int = 128, alpha: float = 1e-5,
              eps: float = 0.001, T: float = 0.5) -> Instance:
    """3D, (0,1)^3, Gaussian bump centre (0.4,0.5,0.6) width 0.1, T=0.5, 0.1% noise."""
    rng = np.random.default_rng(seed)
    x = nodes(m, 1.0)
    # array axes are (x_3, x_2, x_1)
    X3, X2, X1 = np.meshgrid(x, x, x, indexing="ij")
    r2 = (X1 - 0.4) ** 2 + (X2 - 0.5) ** 2 + (X3 - 0.6) ** 2
    z0 = np.exp(-r2 / (2.0 * 0.1 ** 2))
    g = forward_final_state_dense(z0, n, 1.0, T)
    g_delta, delta = add_relative_noise(g, eps, rng, 1.0 / (m + 1))
    return Instance(3, m, n, 1.0, T, alpha, 0, g_delta, delta, z0, g, eps)


def config_batched(seed: int = 3, count_1d: int = 256, count_2d: int = 256,
                   m1d=(63, 1023), m2d=(63, 255), nrange=(64, 512),
                   alpha_log10=(-6.0, -1.0), eps_log10=(-3.0, math.log10(0.05))) -> list:
    """Uneven batch: 1D and 2D sine-mode instances with random m, n, alpha, noise level."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count_1d + count_2d):
        d = 1 if i < count_1d else 2
        lo, hi = m1d if d == 1 else m2d
        m = int(rng.integers(lo, hi + 1))
        n = int(rng.integers(nrange[0], nrange[1] + 1))
        alpha = 10.0 ** rng.uniform(*alpha_log10)
        eps = 10.0 ** rng.uniform(*eps_log10)
        out.append(sine_mode_instance(d, m, n, 1.0, alpha, eps, rng))
    return out


def config_learned(seed: int, count: int, m: int = 127, n: int = 128, T: float = 1.0,
                   eps_log10=(-3.0, math.log10(0.05))):
    """Training / held-out sets for the alpha predictor: 2D sine-mode data, noise 0.1%..5%.

    Returns (g_delta[count, m, m], delta[count], z0[count, m, m], eps[count]).
    Vectorised over instances; per instance the draw order is coefficients, then noise.
    """
    rng = np.random.default_rng(seed)
    modes = _lowest_modes(2, m)
    C = modes.shape[0]
    ksq = np.sum(modes.astype(np.float64) ** 2, axis=1)
    x = nodes(m, 1.0)
    tau = T / n
    lam = _stencil_eig_1d(modes[:, 0].astype(np.float64), m, 1.0) + \
        _stencil_eig_1d(modes[:, 1].astype(np.float64), m, 1.0)
    decay = (1.0 / (1.0 + tau * lam)) ** n
    s1 = np.sin(np.outer(modes[:, 0], x) * np.pi)   # (C, m) x_1 factor
    s2 = np.sin(np.outer(modes[:, 1], x) * np.pi)   # (C, m) x_2 factor
    h = 1.0 / (m + 1)
    gd = np.empty((count, m, m))
    z0s = np.empty((count, m, m))
    deltas = np.empty(count)
    epss = np.empty(count)
    for i in range(count):
        coef = rng.standard_normal(C) / (1.0 + ksq)
        eps = 10.0 ** rng.uniform(*eps_log10)
        z0 = (s2.T * coef) @ s1
        g = (s2.T * (coef * decay)) @ s1
        eta = rng.standard_normal((m, m))
        gn = np.linalg.norm(g)
        gd[i] = g + (eps * gn / np.linalg.norm(eta)) * eta
        z0s[i] = z0
        deltas[i] = eps * gn * h
        epss[i] = eps
    return gd, deltas, z0s, epss
