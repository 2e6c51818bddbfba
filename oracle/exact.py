"""Closed forms and exact discrete solves -- TEST INFRASTRUCTURE ONLY.

These pin the oracle's sweep (``oracle.c``) without reusing it: they follow
from the mathematics of Section IV of the ProtoX paper (the 5-point stencil of
Eq. 1 with the filter taps of the OL Laplace expression, the Poisson problem
of Eq. 2 and the Jacobi step of Eq. 3), not from the sweep's code.

Boundary reading: homogeneous Dirichlet on a cell-centred grid (h = 1/n),
odd reflection ghost = -(adjacent interior).  Under it the cell-centred sine
modes sin(p pi x) sin(q pi y), p, q = 1..n, are exact eigenvectors of the
discrete Laplacian L = S/h^2 with eigenvalues

    mu_pq = -(4/h^2) (sin^2(p pi h/2) + sin^2(q pi h/2)),

so the Jacobi step phi <- phi + lambda (L phi - f) multiplies the error's
(p, q) component by  g_pq = 1 + lambda mu_pq = 1 - omega (sin^2 + sin^2)
with omega = 4 lambda / h^2.  The node-centred variant (zero ghosts held
fixed, h = 1/(n+1), nodes at i h) has the same eigen-structure.
"""
from __future__ import annotations

import numpy as np
from scipy import fft as _fft


def eigenvalues(n: int, h: float, node_centred: bool = False) -> np.ndarray:
    """mu_pq for p, q = 1..n (n x n array, row index p ~ y)."""
    p = np.arange(1, n + 1, dtype=np.float64)
    if node_centred:
        s = np.sin(p * np.pi / (2.0 * (n + 1))) ** 2
    else:
        s = np.sin(p * np.pi / (2.0 * n)) ** 2
    return -(4.0 / (h * h)) * (s[:, None] + s[None, :])


def mode_factor(n: int, p: int, q: int, omega: float, node_centred: bool = False) -> float:
    """Per-sweep damping factor g_pq of the (p, q) error mode."""
    d = 2.0 * (n + 1) if node_centred else 2.0 * n
    return 1.0 - omega * (np.sin(p * np.pi / d) ** 2 + np.sin(q * np.pi / d) ** 2)


def dst_solve(f: np.ndarray, h: float) -> np.ndarray:
    """Exact solution of L phi = f (cell-centred, odd-reflection Dirichlet) by
    diagonalisation in the orthonormal DST-II basis."""
    n = f.shape[0]
    assert f.shape == (n, n)
    fh = _fft.dstn(f, type=2, norm="ortho", workers=-1)
    return _fft.idstn(fh / eigenvalues(n, h), type=2, norm="ortho", workers=-1)


def dense_laplacian(n: int, h: float, node_centred: bool = False) -> np.ndarray:
    """The n^2 x n^2 matrix of L = S/h^2 with the ghost cells eliminated.

    Cell-centred odd reflection: a ghost equal to -(adjacent) adds -1 to the
    diagonal per missing neighbour (-5 on edges, -6 at corners).  Node-centred
    zero ghosts: the missing neighbour simply drops out (-4 everywhere)."""
    N = n * n
    A = np.zeros((N, N), dtype=np.float64)
    for i in range(n):
        for j in range(n):
            k = i * n + j
            A[k, k] = -4.0
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < n and 0 <= jj < n:
                    A[k, ii * n + jj] += 1.0
                elif not node_centred:
                    A[k, k] -= 1.0
    return A / (h * h)


def dense_solve(f: np.ndarray, h: float, node_centred: bool = False) -> np.ndarray:
    n = f.shape[0]
    return np.linalg.solve(dense_laplacian(n, h, node_centred), f.ravel()).reshape(n, n)


def dense_jacobi(phi0: np.ndarray, f: np.ndarray, h: float, lam: float, nsweeps: int,
                 node_centred: bool = False) -> np.ndarray:
    """nsweeps Jacobi steps phi <- phi + lam (A phi - f) with the dense matrix A."""
    n = f.shape[0]
    A = dense_laplacian(n, h, node_centred)
    x = phi0.ravel().copy()
    b = f.ravel()
    for _ in range(nsweeps):
        x = x + lam * (A @ x - b)
    return x.reshape(n, n)


def manufactured_closed_form(n: int, nsweeps: int, omega: float, node_centred: bool = False):
    """Closed form of plain Jacobi from phi0 = 0 for f = -2 pi^2 u, u = sin(pi x) sin(pi y).

    u is the (1,1) eigenmode, so the discrete solution is phi_h = s u with
    s = 2 pi^2 / |mu_11|, the error after N sweeps is -g^N s u and the residual
    is g^N f.  Returns a dict of the quantities the tests compare against."""
    if node_centred:
        h = 1.0 / (n + 1)
        x = (np.arange(n) + 1.0) * h
    else:
        h = 1.0 / n
        x = (np.arange(n) + 0.5) * h
    lam = omega * h * h / 4.0
    g = mode_factor(n, 1, 1, omega, node_centred)
    mu = -(8.0 / (h * h)) * np.sin(np.pi * h / 2.0) ** 2  # mu_11
    s = 2.0 * np.pi ** 2 / (-mu)
    umax = np.max(np.sin(np.pi * x)) ** 2
    fmax = 2.0 * np.pi ** 2 * umax
    u = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
    f = -2.0 * np.pi ** 2 * u
    phiN = s * (1.0 - g ** nsweeps) * u
    return {
        "h": h, "lambda": lam, "w": lam / (h * h), "g": g, "s": s,
        "f_max": fmax,
        "rel_res": g ** nsweeps,
        "res_max_final": g ** nsweeps * fmax,
        "res_max_lagged": g ** (nsweeps - 1) * fmax,
        "res_l2sq_final": g ** (2 * nsweeps) * float(np.sum(f * f)),
        "err_max": abs(s * (1.0 - g ** nsweeps) - 1.0) * umax,
        "err_rms": abs(s * (1.0 - g ** nsweeps) - 1.0) * float(np.sqrt(np.mean(u * u))),
        "phi": phiN,
        "disc_err_max": abs(s - 1.0) * umax,
    }
