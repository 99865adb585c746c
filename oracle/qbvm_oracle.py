"""CPU FP64 oracle for PinT-QBVM / PinT-MQBVM (arXiv 2107.06381).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU-baseline
leg of the benchmark, never by the library.  Plain numpy/scipy in float64.

What is computed, and from which passage:

* The all-at-once system (Section 3.1, the PinT-QBVM scheme and matrix \\hat A_h;
  Section 3.2, the PinT-MQBVM scheme and \\hat B_h).  Rows, for every interior
  node p (x_1 fastest) and level t:
      t = 0 :  (1/tau) y^0_p - (Lap_h y^0)_p - (omega/tau) y^N_p = f0_p
      t >= 1:  (1/tau) y^t_p - (Lap_h y^t)_p - (1/tau) y^{t-1}_p = 0
  with omega = -1/alpha, f0 = g/(tau alpha) (PinT-QBVM) or omega = -tau/alpha,
  f0 = g/alpha (PinT-MQBVM).  The solution is y_h = A^{-1} f: the PinT solver is
  a direct method, so its exact output is this solution.
  - ``assemble_allatonce`` writes these rows out one equation at a time.
  - ``solve_dense`` (LAPACK LU) and ``solve_splu`` (SuperLU) solve them.
* The per-eigenmode closed form (``closed_form``): the rows decouple in the
  orthonormal sine basis of the Dirichlet stencil.  Per mode with eigenvalue mu
  of -Lap_h and r = 1/(1+tau mu): y^t = r^t y^0 and
      y^0 = f0_hat / ((1/tau + mu) - (omega/tau) r^N),
  the discrete counterpart of the series representations of Section 4.
* The paper's three-step diagonalisation solver (Section 3.3, eq. "3step") in
  dense form for tiny sizes (``pint_three_step``), with the explicit
  omega-circulant eigen-decomposition C = V D V^{-1}, V = Gamma^{-1} F^*.
* The residual of the all-at-once rows, matrix free (``residual``).
* The same rows with another spatial matrix A in place of -Lap_h (Section 3.3: the
  operator enters only Step (b)): a general tridiagonal A in 1D, and in 2D the
  variable-coefficient diffusion -div(kappa grad u) in conservative five-point form
  (``diffusion_matrix_2d``) and its seven-point 3D counterpart (``diffusion_matrix_3d``); solved by ``solve_splu_operator`` (SuperLU) and
  ``closed_form_operator`` (eigenbasis of A), with the matrix-free residual
  ``residual_operator`` for sizes beyond either.
* Discrepancy-principle quantities and the bisection used to label alpha, the
  spectral features of g_delta (``discrepancy``, ``bisect_alpha``, ``features``);
  these are additions not taken from the paper, see their docstrings.

Readings where the paper is silent (grid, norm, ordering) are listed in the design
notes; in short: h = L/(m+1), tau = T/n, N_t = n+1, arrays are (t, x_d, ..., x_1)
in C order, ||v||_h = h^{d/2} ||v||_2.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

PQ = 0  # PinT-QBVM  (Section 3.1)
PM = 1  # PinT-MQBVM (Section 3.2)


# ----------------------------------------------------------------------------
# grid and scheme constants (Section 2: tau = T/N, h = L/M; N_t = N+1)
# ----------------------------------------------------------------------------
def grid_constants(d: int, m: int, n: int, L: float, T: float):
    h = L / (m + 1)
    tau = T / n
    return h, tau, n + 1, m ** d


def omega_and_scale(alpha: float, variant: int, tau: float):
    """omega and the factor f0 = scale * g (Sections 3.1 and 3.2)."""
    if variant == PQ:
        return -1.0 / alpha, 1.0 / (tau * alpha)
    if variant == PM:
        return -tau / alpha, 1.0 / alpha
    raise ValueError("variant must be 0 (PinT-QBVM) or 1 (PinT-MQBVM)")


def stencil_eigenvalues(d: int, m: int, L: float) -> np.ndarray:
    """Eigenvalues mu_k of -Lap_h on the sine modes, shape (m,)*d in (x_d..x_1) order.

    1D textbook result for the 3-point Dirichlet stencil: (4/h^2) sin^2(k pi/(2(m+1))),
    summed over the dimensions for the (2d+1)-point stencil.
    """
    h = L / (m + 1)
    k = np.arange(1, m + 1, dtype=np.float64)
    mu1 = (4.0 / h ** 2) * np.sin(k * np.pi / (2.0 * (m + 1))) ** 2
    mu = np.zeros((m,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = m
        mu = mu + mu1.reshape(shape)
    return mu


def dst_ortho(x: np.ndarray) -> np.ndarray:
    """Orthonormal type-I DST over every axis (symmetric and its own inverse)."""
    return sfft.dstn(x, type=1, norm="ortho")


# ----------------------------------------------------------------------------
# O1 / O2: the all-at-once system, assembled row by row
# ----------------------------------------------------------------------------
def _node_neighbours(d: int, m: int):
    """For every interior node p (x_1 fastest): list of (p, q) neighbour pairs."""
    idx = np.arange(m ** d).reshape((m,) * d)
    pairs = []
    for ax in range(d):
        lo = [slice(None)] * d
        hi = [slice(None)] * d
        lo[ax] = slice(0, m - 1)
        hi[ax] = slice(1, m)
        a = idx[tuple(lo)].ravel()
        b = idx[tuple(hi)].ravel()
        pairs.append(np.stack([a, b], 1))
        pairs.append(np.stack([b, a], 1))
    return np.concatenate(pairs, 0) if pairs else np.zeros((0, 2), np.int64)


def assemble_allatonce(d: int, m: int, n: int, L: float, T: float, alpha: float,
                       variant: int) -> sp.csr_matrix:
    """Sparse matrix of the PinT system: one block row per time level (eq. 3.x rows)."""
    h, tau, Nt, Nx = grid_constants(d, m, n, L, T)
    omega, _ = omega_and_scale(alpha, variant, tau)
    nb = _node_neighbours(d, m)
    rows, cols, vals = [], [], []
    diag = 1.0 / tau + 2.0 * d / h ** 2
    p = np.arange(Nx)
    for t in range(Nt):
        base = t * Nx
        # (1/tau) y^t - Lap_h y^t : diagonal and the stencil neighbours
        rows.append(base + p); cols.append(base + p); vals.append(np.full(Nx, diag))
        rows.append(base + nb[:, 0]); cols.append(base + nb[:, 1])
        vals.append(np.full(nb.shape[0], -1.0 / h ** 2))
        if t == 0:
            # -(omega/tau) y^N in the first block row
            rows.append(base + p); cols.append((Nt - 1) * Nx + p)
            vals.append(np.full(Nx, -omega / tau))
        else:
            # -(1/tau) y^{t-1}
            rows.append(base + p); cols.append((t - 1) * Nx + p)
            vals.append(np.full(Nx, -1.0 / tau))
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(Nt * Nx, Nt * Nx))
    return A


def rhs_allatonce(g_delta: np.ndarray, n: int, alpha: float, variant: int, T: float):
    tau = T / n
    _, scale = omega_and_scale(alpha, variant, tau)
    Nx = g_delta.size
    f = np.zeros((n + 1) * Nx)
    f[:Nx] = scale * np.ravel(g_delta)
    return f


def solve_dense(g_delta, d, m, n, L, T, alpha, variant):
    """O1: dense LU (numpy.linalg.solve) of the assembled system; tiny sizes only."""
    A = assemble_allatonce(d, m, n, L, T, alpha, variant).toarray()
    f = rhs_allatonce(g_delta, n, alpha, variant, T)
    return np.linalg.solve(A, f).reshape((n + 1,) + (m,) * d)


def solve_splu(g_delta, d, m, n, L, T, alpha, variant):
    """O2: sparse LU (SuperLU, COLAMD ordering) of the assembled system."""
    A = assemble_allatonce(d, m, n, L, T, alpha, variant).tocsc()
    f = rhs_allatonce(g_delta, n, alpha, variant, T)
    lu = spla.splu(A, permc_spec="COLAMD")
    return lu.solve(f).reshape((n + 1,) + (m,) * d)


def solve_general_splu(f, d, m, n, L, T, alpha, variant):
    """O2 for a general right-hand side f (one block per level, shape (n+1,)+(m,)*d):
    A y = f with the assembled all-at-once matrix (Sections 3.1, 3.2), by sparse LU.
    This is one source-term solve, or one application of the PinT system as a
    preconditioner (mentioned at the end of Section 2 and in Section 5)."""
    A = assemble_allatonce(d, m, n, L, T, alpha, variant).tocsc()
    lu = spla.splu(A, permc_spec="COLAMD")
    return lu.solve(np.ravel(np.asarray(f, dtype=np.float64))).reshape((n + 1,) + (m,) * d)


def closed_form_general(f, d, m, n, L, T, alpha, variant):
    """O3 for a general right-hand side: in the sine basis every mode k obeys the scheme
    rows (1/tau + mu_k) y^t - y^{t-1}/tau = f^t_k (t >= 1) and
    (1/tau + mu_k) y^0 - (omega/tau) y^N = f^0_k.  With r = 1/(1 + tau mu_k) the march
    gives y^t = r y^{t-1} + tau r f^t, so y^N = r^N y^0 + P with
    P = sum_{t>=1} r^{N-t} tau r f^t; the first row then fixes y^0 and the march the rest."""
    h, tau, Nt, _ = grid_constants(d, m, n, L, T)
    omega, _ = omega_and_scale(alpha, variant, tau)
    mu = stencil_eigenvalues(d, m, L)
    r = 1.0 / (1.0 + tau * mu)
    fh = np.stack([dst_ortho(np.asarray(f[t], dtype=np.float64)) for t in range(Nt)], 0)
    P = np.zeros_like(mu)
    for t in range(1, Nt):
        P = r * P + tau * r * fh[t]
    y = np.empty_like(fh)
    y[0] = (fh[0] + (omega / tau) * P) / ((1.0 / tau + mu) - (omega / tau) * r ** n)
    for t in range(1, Nt):
        y[t] = r * y[t - 1] + tau * r * fh[t]
    return np.stack([dst_ortho(y[t]) for t in range(Nt)], 0)


# ----------------------------------------------------------------------------
# O3: per-eigenmode closed form
# ----------------------------------------------------------------------------
def closed_form_spectral(g_hat, d, m, n, L, T, alpha, variant, levels=None):
    """Mode amplitudes y^t_k (sine basis) for the requested levels (default all)."""
    h, tau, Nt, _ = grid_constants(d, m, n, L, T)
    omega, scale = omega_and_scale(alpha, variant, tau)
    mu = stencil_eigenvalues(d, m, L)
    r = 1.0 / (1.0 + tau * mu)
    y0 = scale * g_hat / ((1.0 / tau + mu) - (omega / tau) * r ** n)
    if levels is None:
        levels = range(Nt)
    return np.stack([y0 * r ** t for t in levels], 0)


def closed_form(g_delta, d, m, n, L, T, alpha, variant, levels=None):
    """O3: y^t on the grid, shape (len(levels),) + (m,)*d."""
    g_hat = dst_ortho(np.asarray(g_delta, dtype=np.float64))
    yk = closed_form_spectral(g_hat, d, m, n, L, T, alpha, variant, levels)
    axes = tuple(range(1, d + 1))
    return sfft.idstn(yk, type=1, norm="ortho", axes=axes)


# ----------------------------------------------------------------------------
# the paper's three-step solver, dense, tiny sizes (Section 3.3)
# ----------------------------------------------------------------------------
def circulant_matrix(omega: float, Nt: int) -> np.ndarray:
    """C_omega: 1 on the diagonal, -1 on the subdiagonal, -omega in the top-right corner."""
    C = np.eye(Nt) - np.eye(Nt, k=-1)
    C[0, Nt - 1] = -omega
    return C


def circulant_factors(omega: float, Nt: int):
    """F, Gamma_omega and D of the explicit diagonalisation C = V D V^{-1}.

    F = (1/sqrt(N_t)) [theta^{(l1-1)(l2-1)}], theta = exp(2 pi i/N_t);
    Gamma = diag(omega^{l/N_t}) with the principal root of the negative omega;
    D = diag(sqrt(N_t) F Gamma C(:,1)).
    """
    l = np.arange(Nt)
    F = np.exp(2j * np.pi * np.outer(l, l) / Nt) / math.sqrt(Nt)
    root = np.exp((math.log(abs(omega)) + (1j * math.pi if omega < 0 else 0.0)) / Nt)
    gam = root ** l
    C = circulant_matrix(omega, Nt)
    Dv = math.sqrt(Nt) * (F @ (gam * C[:, 0]))
    return F, gam, Dv


def laplacian_matrix(d: int, m: int, L: float) -> sp.csr_matrix:
    """Lap_h (negative semidefinite), (2d+1)-point Dirichlet stencil, x_1 fastest."""
    h = L / (m + 1)
    Nx = m ** d
    nb = _node_neighbours(d, m)
    rows = np.concatenate([np.arange(Nx), nb[:, 0]])
    cols = np.concatenate([np.arange(Nx), nb[:, 1]])
    vals = np.concatenate([np.full(Nx, -2.0 * d / h ** 2), np.full(nb.shape[0], 1.0 / h ** 2)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(Nx, Nx))


# ----------------------------------------------------------------------------
# Another spatial operator (1D): Section 3.3 notes that the diagonalisation in time
# is independent of the spatial operator, which enters only through Step (b).  A is
# a general m x m tridiagonal matrix standing in for -Lap_h in every block row.
# ----------------------------------------------------------------------------
def tridiagonal_matrix(lower, diag, upper) -> sp.csr_matrix:
    """A with A[i, i-1] = lower[i-1], A[i, i] = diag[i], A[i, i+1] = upper[i]."""
    m = len(diag)
    return sp.diags([np.asarray(lower, float), np.asarray(diag, float), np.asarray(upper, float)],
                    [-1, 0, 1], shape=(m, m), format="csr")


def assemble_allatonce_operator(A, n: int, T: float, alpha: float, variant: int) -> sp.csr_matrix:
    """The rows of Sections 3.1/3.2 with A in place of -Lap_h:
    t = 0: (I/tau + A) y^0 - (omega/tau) y^N = f0;  t >= 1: (I/tau + A) y^t - y^{t-1}/tau = 0."""
    tau = T / n
    Nt = n + 1
    omega, _ = omega_and_scale(alpha, variant, tau)
    Nx = A.shape[0]
    Ix = sp.identity(Nx, format="csr")
    It = sp.identity(Nt, format="csr")
    back = sp.diags([np.ones(Nt - 1)], [-1], shape=(Nt, Nt), format="csr")   # (t, t-1)
    corner = sp.csr_matrix(([1.0], ([0], [Nt - 1])), shape=(Nt, Nt))          # (0, N)
    return (sp.kron(It, Ix / tau + A) - sp.kron(back, Ix) / tau - (omega / tau) * sp.kron(corner, Ix)).tocsr()


def solve_splu_operator(g_delta, A, n: int, T: float, alpha: float, variant: int):
    """O2 with the operator A: SuperLU on the assembled rows; (n+1, m) levels."""
    M = assemble_allatonce_operator(A, n, T, alpha, variant).tocsc()
    f = rhs_allatonce(np.asarray(g_delta, float), n, alpha, variant, T)
    return spla.splu(M, permc_spec="COLAMD").solve(f).reshape(n + 1, -1)


def closed_form_operator(g_delta, A, n: int, T: float, alpha: float, variant: int):
    """O3 with the operator A: in the eigenbasis of A (A = U diag(lam) U^{-1}; LAPACK eigh
    when A is symmetric, eig otherwise) every mode obeys the closed form of the Dirichlet
    case with mu -> lam: y^t = r^t y^0, r = 1/(1 + tau lam),
    y^0 = f0_hat / ((1/tau + lam) - (omega/tau) r^N).  Returns the real part."""
    tau = T / n
    omega, scale = omega_and_scale(alpha, variant, tau)
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A, float)
    f0 = scale * np.ravel(np.asarray(g_delta, float))
    if np.array_equal(Ad, Ad.T):
        lam, U = np.linalg.eigh(Ad)
        fh = U.T @ f0
    else:
        lam, U = np.linalg.eig(Ad)
        fh = np.linalg.solve(U, f0.astype(complex))
    r = 1.0 / (1.0 + tau * lam)
    y0 = fh / ((1.0 / tau + lam) - (omega / tau) * r ** n)
    modes = y0[:, None] * r[:, None] ** np.arange(n + 1)[None, :]   # [mode][t] = r^t y^0
    return np.ascontiguousarray(np.real(U @ modes).T)


def diffusion_matrix_2d(kx, ky, L: float) -> sp.csr_matrix:
    """-div(kappa grad u) on the m x m interior grid with zero Dirichlet data, in the
    conservative five-point form with kappa at the cell faces (kx: (m, m+1) faces
    between x_1 neighbours, ky: (m+1, m) faces between x_2 neighbours; node (j, i) is
    x_1 = (i+1) h, x_2 = (j+1) h, flattened x_1 fastest):
        (A u)_{j,i} = [kx_{j,i} (u_{j,i} - u_{j,i-1}) + kx_{j,i+1} (u_{j,i} - u_{j,i+1})
                     + ky_{j,i} (u_{j,i} - u_{j-1,i}) + ky_{j+1,i} (u_{j,i} - u_{j+1,i})] / h^2,
    u = 0 outside the grid.  kappa = 1 gives -Lap_h.  Written out one node at a time."""
    kx = np.asarray(kx, float)
    ky = np.asarray(ky, float)
    m = kx.shape[0]
    if kx.shape != (m, m + 1) or ky.shape != (m + 1, m):
        raise ValueError("kx must be (m, m+1) and ky (m+1, m)")
    ih2 = 1.0 / (L / (m + 1)) ** 2
    rows, cols, vals = [], [], []
    for j in range(m):
        for i in range(m):
            p = j * m + i
            rows.append(p)
            cols.append(p)
            vals.append((kx[j, i] + kx[j, i + 1] + ky[j, i] + ky[j + 1, i]) * ih2)
            for (jj, ii, kap) in ((j, i - 1, kx[j, i]), (j, i + 1, kx[j, i + 1]),
                                  (j - 1, i, ky[j, i]), (j + 1, i, ky[j + 1, i])):
                if 0 <= jj < m and 0 <= ii < m:
                    rows.append(p)
                    cols.append(jj * m + ii)
                    vals.append(-kap * ih2)
    return sp.csr_matrix((vals, (rows, cols)), shape=(m * m, m * m))


def diffusion_matrix_3d(kx, ky, kz, L: float) -> sp.csr_matrix:
    """The same conservative form in 3D: node (k, j, i) at x_1 = (i+1) h, x_2 = (j+1) h,
    x_3 = (k+1) h, flattened x_1 fastest; kx (m, m, m+1) faces between x_1 neighbours,
    ky (m, m+1, m) between x_2 neighbours, kz (m+1, m, m) between x_3 neighbours:
        (A u)_{k,j,i} = sum over the six faces of kappa_face (u_{k,j,i} - u_neighbour) / h^2,
    u = 0 outside the grid.  Written out one node at a time."""
    kx = np.asarray(kx, float)
    ky = np.asarray(ky, float)
    kz = np.asarray(kz, float)
    m = kx.shape[0]
    if kx.shape != (m, m, m + 1) or ky.shape != (m, m + 1, m) or kz.shape != (m + 1, m, m):
        raise ValueError("kx must be (m, m, m+1), ky (m, m+1, m) and kz (m+1, m, m)")
    ih2 = 1.0 / (L / (m + 1)) ** 2
    rows, cols, vals = [], [], []
    for k in range(m):
        for j in range(m):
            for i in range(m):
                p = (k * m + j) * m + i
                faces = ((k, j, i - 1, kx[k, j, i]), (k, j, i + 1, kx[k, j, i + 1]),
                         (k, j - 1, i, ky[k, j, i]), (k, j + 1, i, ky[k, j + 1, i]),
                         (k - 1, j, i, kz[k, j, i]), (k + 1, j, i, kz[k + 1, j, i]))
                rows.append(p)
                cols.append(p)
                vals.append(sum(f[3] for f in faces) * ih2)
                for (kk, jj, ii, kap) in faces:
                    if 0 <= kk < m and 0 <= jj < m and 0 <= ii < m:
                        rows.append(p)
                        cols.append((kk * m + jj) * m + ii)
                        vals.append(-kap * ih2)
    return sp.csr_matrix((vals, (rows, cols)), shape=(m ** 3, m ** 3))


def residual_operator(y, g_delta, A, n: int, T: float, alpha: float, variant: int) -> float:
    """||f - M y|| / ||f|| for the rows of Sections 3.1/3.2 with the operator A, applied
    level by level (M never formed): t = 0: (I/tau + A) y^0 - (omega/tau) y^N;
    t >= 1: (I/tau + A) y^t - y^{t-1}/tau.  y: (n+1, m^d) levels."""
    tau = T / n
    omega, scale = omega_and_scale(alpha, variant, tau)
    Y = np.asarray(y, float).reshape(n + 1, -1)
    R = Y / tau + (A @ Y.T).T
    R[0] -= (omega / tau) * Y[n]
    R[1:] -= Y[:-1] / tau
    f0 = scale * np.ravel(np.asarray(g_delta, float))
    R[0] -= f0
    return float(np.linalg.norm(R) / np.linalg.norm(f0))


def pint_three_step(g_delta, d, m, n, L, T, alpha, variant):
    """Steps (a)-(c) of eq. "3step" with dense V, V^{-1} and sparse solves per column."""
    h, tau, Nt, Nx = grid_constants(d, m, n, L, T)
    omega, scale = omega_and_scale(alpha, variant, tau)
    F, gam, Dv = circulant_factors(omega, Nt)
    Vinv = F @ np.diag(gam)                    # V^{-1} = F Gamma
    V = np.diag(1.0 / gam) @ F.conj().T        # V = Gamma^{-1} F^*
    Fhat = np.zeros((Nx, Nt))
    Fhat[:, 0] = scale * np.ravel(g_delta)    # mat(f_h): column j = level j
    S1 = Fhat @ Vinv.T                         # Step (a)
    Lap = laplacian_matrix(d, m, L).tocsc()
    I = sp.identity(Nx, format="csc")
    S2 = np.empty_like(S1)
    for j in range(Nt):                        # Step (b)
        S2[:, j] = spla.spsolve((Dv[j] / tau) * I - Lap, S1[:, j])
    Y = S2 @ V.T                               # Step (c)
    return Y.T.reshape((Nt,) + (m,) * d), Y


# ----------------------------------------------------------------------------
# O4: residual of the all-at-once rows (matrix free)
# ----------------------------------------------------------------------------
def apply_laplacian(y: np.ndarray, h: float) -> np.ndarray:
    """Lap_h applied to every level of y (shape (Nt,)+(m,)*d), zero Dirichlet data."""
    d = y.ndim - 1
    out = -2.0 * d * y
    for ax in range(1, d + 1):
        sl_lo = [slice(None)] * y.ndim
        sl_hi = [slice(None)] * y.ndim
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        out[tuple(sl_hi)] += y[tuple(sl_lo)]
        out[tuple(sl_lo)] += y[tuple(sl_hi)]
    return out / h ** 2


def residual(y, g_delta, d, m, n, L, T, alpha, variant) -> float:
    """||f - A y|| / ||f|| with A applied row by row from the scheme."""
    h, tau, Nt, _ = grid_constants(d, m, n, L, T)
    omega, scale = omega_and_scale(alpha, variant, tau)
    Ay = y / tau - apply_laplacian(y, h)
    Ay[0] -= (omega / tau) * y[Nt - 1]
    Ay[1:] -= y[:-1] / tau
    f = np.zeros_like(y)
    f[0] = scale * g_delta
    return float(np.linalg.norm((f - Ay).ravel()) / np.linalg.norm(f.ravel()))


# ----------------------------------------------------------------------------
# discrepancy principle (addition, not from the paper)
# ----------------------------------------------------------------------------
def discrepancy(alpha, g_delta, d, m, n, L, T, variant=PQ, g_hat=None) -> float:
    """D(alpha) = ||y^N(alpha) - g_delta||_h, evaluated in the sine basis (Parseval)."""
    h = L / (m + 1)
    if g_hat is None:
        g_hat = dst_ortho(np.asarray(g_delta, dtype=np.float64))
    yN = closed_form_spectral(g_hat, d, m, n, L, T, alpha, variant, levels=[n])[0]
    return float(h ** (d / 2.0) * np.linalg.norm((yN - g_hat).ravel()))


def bisect_alpha(g_delta, delta, d, m, n, L, T, variant=PQ, tau_dp=1.1,
                 log10_lo=-20.0, log10_hi=0.0, steps=30):
    """30 halvings of log10(alpha) for D(alpha) = tau_dp * delta.

    D is increasing in alpha: if D(10^mid) > tau_dp*delta the root is below mid.
    Returns (alpha, bracket_hit) with alpha = 10^((lo+hi)/2) of the final bracket;
    bracket_hit is 1 if the root lies outside [lo, hi] (the nearer end is returned).
    """
    h = L / (m + 1)
    g_hat = dst_ortho(np.asarray(g_delta, dtype=np.float64))
    target = tau_dp * delta
    lo, hi = float(log10_lo), float(log10_hi)
    if discrepancy(10.0 ** hi, g_delta, d, m, n, L, T, variant, g_hat) <= target:
        return 10.0 ** hi, 1
    if discrepancy(10.0 ** lo, g_delta, d, m, n, L, T, variant, g_hat) > target:
        return 10.0 ** lo, 1
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if discrepancy(10.0 ** mid, g_delta, d, m, n, L, T, variant, g_hat) > target:
            hi = mid
        else:
            lo = mid
    return 10.0 ** (0.5 * (lo + hi)), 0


# ----------------------------------------------------------------------------
# learned-alpha features (addition, not from the paper)
# ----------------------------------------------------------------------------
NBINS = 32


def feature_bins(d: int, m: int) -> np.ndarray:
    """Bin of every sine mode: 32 equal-width bins of rho = |k|_2 over [sqrt(d), m sqrt(d)]."""
    k = np.arange(1, m + 1, dtype=np.float64)
    ksq = np.zeros((m,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = m
        ksq = ksq + (k ** 2).reshape(shape)
    rho = np.sqrt(ksq)
    lo = math.sqrt(d)
    hi = m * math.sqrt(d)
    if m == 1:
        return np.zeros((1,) * d, dtype=np.int64)
    t = (rho - lo) / (hi - lo) * NBINS
    b = np.floor(t).astype(np.int64)
    return np.clip(b, 0, NBINS - 1)


def features(g_delta: np.ndarray, delta: float, L: float = 1.0) -> np.ndarray:
    """33 features: log10 of the h^d-weighted sine-spectrum energy in each bin, and log10 delta."""
    d = g_delta.ndim
    m = g_delta.shape[0]
    h = L / (m + 1)
    gh = dst_ortho(np.asarray(g_delta, dtype=np.float64))
    b = feature_bins(d, m).ravel()
    e = np.bincount(b, weights=(gh.ravel() ** 2), minlength=NBINS) * h ** d
    return np.concatenate([np.log10(e + 1e-300), [math.log10(delta)]])


def reconstruction_error(y0, z0, L: float = 1.0) -> float:
    """e_h = ||y^0 - z(.,0)||_h (Section 5)."""
    d = z0.ndim
    h = L / (z0.shape[0] + 1)
    return float(h ** (d / 2.0) * np.linalg.norm((y0 - z0).ravel()))
