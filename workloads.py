"""Seeded synthetic inputs for the 2D Poisson relaxation.

This module only produces input arrays (right-hand sides, initial iterates and
problem-size lists).  It holds none of the method's arithmetic: no stencil,
sweep, residual or norm.  Both the CPU oracle's tests and the GPU path draw
their inputs from here, so the two see identical data.

Conventions (Section IV of the ProtoX paper, "2D Poisson equation"): the
domain is the unit square, an n x n grid of cells with spacing h = 1/n, cell
centres at ((j + 1/2) h, (i + 1/2) h) for row i and column j, row-major, the
column index fastest.  Every generator returns float64 arrays; callers cast.
"""
from __future__ import annotations

import numpy as np
from scipy import fft as _fft

# Seeds of the named workloads (recorded in benchmark output).
SEED_UNIFORM_4096 = 2
SEED_GRF_8192 = 3
SEED_BATCH_SIZES = 4
SEED_BATCH_BASE = 4000
SEED_TRAIN_BASE = 5000
SEED_EVAL_BASE = 9000

BATCH_SIZE_CHOICES = (64, 128, 256, 512, 1024)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def cell_centres(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def manufactured_rhs(n: int) -> np.ndarray:
    """f = -2 pi^2 sin(pi x) sin(pi y) at cell centres (the right-hand side whose
    continuous solution is u = sin(pi x) sin(pi y))."""
    x = cell_centres(n)
    s = np.sin(np.pi * x)
    return -2.0 * np.pi ** 2 * np.outer(s, s)


def manufactured_solution(n: int) -> np.ndarray:
    x = cell_centres(n)
    s = np.sin(np.pi * x)
    return np.outer(s, s)


def uniform_rhs(n: int, seed: int) -> np.ndarray:
    """f ~ Uniform[-1, 1) i.i.d., row-major, from PCG64(seed)."""
    return rng(seed).uniform(-1.0, 1.0, size=(n, n))


def grf_field(n: int, seed: int, power: float) -> np.ndarray:
    """Gaussian random field with amplitude spectrum |k|^-power in the cell-centred
    sine basis: sum_pq xi_pq |k_pq|^-power sin(p pi x) sin(q pi y), xi ~ N(0,1) from
    PCG64(seed), p, q = 1..n (orthonormal DST-II synthesis), normalised to unit
    root-mean-square.  It vanishes at the cell faces of the boundary in the sense of
    the sine basis."""
    xi = rng(seed).standard_normal(size=(n, n))
    p = np.arange(1, n + 1, dtype=np.float64)
    k2 = p[:, None] ** 2 + p[None, :] ** 2
    amp = 1.0 / np.sqrt(k2) if power == 1.0 else k2 ** (-0.5 * power)
    f = _fft.idstn(xi * amp, type=2, norm="ortho", workers=-1)
    f /= np.sqrt(np.mean(f * f))
    return f


def grf_rhs(n: int, seed: int) -> np.ndarray:
    """Right-hand side with power spectrum ~ |k|^-2 (amplitude |k|^-1): grf_field with
    power 1."""
    return grf_field(n, seed, 1.0)


def error_field(n: int, seed: int) -> np.ndarray:
    """Initial error of a training solve: amplitude spectrum |k|^-3, the spectrum of the
    solution of L u = f for f from grf_rhs (the Laplacian's symbol grows as |k|^2)."""
    return grf_field(n, seed, 3.0)


def sine_mode(n: int, p: int, q: int, node_centred: bool = False) -> np.ndarray:
    """sin(p pi y) sin(q pi x) on the n x n grid (row index ~ y, column ~ x).
    Cell-centred: x_j = (j + 1/2)/n.  Node-centred: x_j = (j + 1)/(n + 1)."""
    if node_centred:
        x = (np.arange(n, dtype=np.float64) + 1.0) / (n + 1)
    else:
        x = cell_centres(n)
    return np.outer(np.sin(p * np.pi * x), np.sin(q * np.pi * x))


def quadratic_grid(n: int, a: int, b: int, c: int, d: int, e: int, g: int,
                   shift: int = 0) -> np.ndarray:
    """(n+2) x (n+2) array of the integer quadratic
    a i^2 + b i j + c j^2 + d i + e j + g at padded indices (i, j), with
    i, j measured from `shift` (ghost ring included)."""
    i = np.arange(n + 2, dtype=np.float64)[:, None] - shift
    j = np.arange(n + 2, dtype=np.float64)[None, :] - shift
    return a * i * i + b * i * j + c * j * j + d * i + e * j + g


def uniform_phi(n: int, seed: int) -> np.ndarray:
    """A random (n+2) x (n+2) iterate, ghost ring included (for parity tests)."""
    return rng(seed).uniform(-1.0, 1.0, size=(n + 2, n + 2))


def batch_sizes(count: int = 512, seed: int = SEED_BATCH_SIZES) -> np.ndarray:
    """Square problem sizes drawn uniformly from {64, 128, 256, 512, 1024}."""
    idx = rng(seed).integers(0, len(BATCH_SIZE_CHOICES), size=count)
    return np.asarray(BATCH_SIZE_CHOICES, dtype=np.int64)[idx]


def embed(interior_or_full: np.ndarray, n: int, ld: int, dtype=np.float64) -> np.ndarray:
    """Place an n x n interior (zero ghost ring) or a full (n+2) x (n+2) grid into
    an (n+2) x ld row-major array; padding columns are zero."""
    out = np.zeros((n + 2, ld), dtype=dtype)
    a = np.asarray(interior_or_full)
    if a.shape == (n, n):
        out[1:n + 1, 1:n + 1] = a
    elif a.shape == (n + 2, n + 2):
        out[:, :n + 2] = a
    else:
        raise ValueError(f"expected ({n},{n}) or ({n + 2},{n + 2}), got {a.shape}")
    return out


def pad_rows(f: np.ndarray, ld_f: int, dtype=np.float64) -> np.ndarray:
    """n x n right-hand side into an n x ld_f row-major array (padding zero)."""
    n = f.shape[0]
    out = np.zeros((n, ld_f), dtype=dtype)
    out[:, :f.shape[1]] = f
    return out


NET_SHAPES = ((32, 1, 3, 3), (32, 32, 3, 3), (32, 32, 3, 3), (1, 32, 3, 3))


def net_initial_weights(seed: int) -> np.ndarray:
    """Initial weights of the 4-layer 3x3 correction network (19008 numbers, layers in
    order, each in (out, in, 3, 3) C order): He-normal, std sqrt(2 / (9 * in)), from
    PCG64(seed)."""
    g = rng(seed)
    return np.concatenate([(g.standard_normal(s) * np.sqrt(2.0 / (s[1] * 9))).ravel() for s in NET_SHAPES])
