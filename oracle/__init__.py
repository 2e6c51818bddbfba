"""CPU oracle for the fused Poisson relaxation -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The product library never loads it,
and it shares no code with the HIP path.

Two parts:

* ``liboracle.so`` (built from ``oracle.c``): the plain three-step sweep of the
  paper's Algorithm (Laplacian, Jacobi update, max-norm; Section IV, Eqs. 1-3
  and the OL expressions for Jacobi and the max-norm), in FP64 with FP32 and
  BF16-storage variants, plus FP64 iterative refinement around the
  low-precision sweep.  Wrapped below with numpy arrays.
* ``exact.py``: closed forms and exact discrete solves (DST-II diagonalisation
  and a dense brute-force solve) that pin the sweep without reusing it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

BC_DIRICHLET0 = 0
BC_GHOST_FIXED = 1
BC_PERIODIC = 2
RES_NONE, RES_LAGGED, RES_FINAL = 0, 1, 2

LAPLACE_TAPS = (0.0, 1.0, 0.0, 1.0, -4.0, 1.0, 0.0, 1.0, 0.0)


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain -O2, no FMA contraction, OpenMP row loops)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-Wall", "-fPIC",
               "-shared", _SRC, "-o", _SO + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        for suf in ("f64", "f32", "bf16"):
            getattr(L, f"ox_apply_stencil_{suf}").argtypes = [P, I, I, P, D, I, P, I]
            getattr(L, f"ox_residual_{suf}").argtypes = [P, I, I, P, I, D, I, P, I, P]
            getattr(L, f"ox_residual_terms_{suf}").argtypes = [P, I, I, P, I, D, I, P, P]
            getattr(L, f"ox_sweep_{suf}").argtypes = [P, P, I, I, P, I, D, D, I, P]
            getattr(L, f"ox_relax_{suf}").argtypes = [P, P, I, I, P, I, D, D, I, I, I, P]
            getattr(L, f"ox_relax_sides_{suf}").argtypes = [P, P, I, I, P, I, D, D, I, P, I, P]
            for nm in ("apply_stencil", "residual", "residual_terms", "sweep", "relax", "relax_sides"):
                getattr(L, f"ox_{nm}_{suf}").restype = None
        L.ox_refine.argtypes = [P, I, I, P, I, D, D, I, I, I, I, D, P]
        L.ox_refine.restype = I
        L.ox_f32_to_bf16.argtypes = [ctypes.c_float]
        L.ox_f32_to_bf16.restype = ctypes.c_uint16
        L.ox_bf16_to_f32.argtypes = [ctypes.c_uint16]
        L.ox_bf16_to_f32.restype = ctypes.c_float
        L.ox_f32_to_bf16_array.argtypes = [P, P, ctypes.c_size_t]
        L.ox_f32_to_bf16_array.restype = None
        L.ox_set_threads.argtypes = [I]
        L.ox_set_threads.restype = None
        L.ox_get_threads.restype = I
        L.ox_max_threads.restype = I
        L.ox_set_threads(default_threads())
        _lib = L
    return _lib


def default_threads() -> int:
    """Threads for the oracle's row loops: the CPUs this process may run on, at most 16
    (one GPU's share of a multi-GPU host)."""
    try:
        cpus = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        cpus = os.cpu_count() or 1
    return max(1, min(16, cpus))


def set_threads(t: int) -> None:
    """Threads of the row loops.  Results do not depend on it: the parallel loops write
    disjoint rows and reduce nothing (the sum of squares stays one sequential loop)."""
    lib().ox_set_threads(int(t))


def get_threads() -> int:
    return int(lib().ox_get_threads())


_SUFFIX = {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32", np.dtype(np.uint16): "bf16"}


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _suffix(a: np.ndarray) -> str:
    try:
        return _SUFFIX[a.dtype]
    except KeyError:
        raise TypeError(f"oracle storage dtype must be float64, float32 or uint16(bf16), got {a.dtype}")


def _check_phi(phi: np.ndarray, n: int):
    assert phi.ndim == 2 and phi.shape[0] == n + 2 and phi.shape[1] >= n + 2, phi.shape
    assert phi.flags.c_contiguous


def _check_f(f: np.ndarray, n: int):
    assert f.ndim == 2 and f.shape[0] == n and f.shape[1] >= n, f.shape
    assert f.flags.c_contiguous


def apply_stencil(phi, n, taps=LAPLACE_TAPS, scale=1.0, bc=BC_DIRICHLET0):
    """out = scale * S(phi) over the n x n interior (Eq. 1, 3x3 taps)."""
    _check_phi(phi, n)
    out = np.zeros((n, n), dtype=phi.dtype)
    t = np.ascontiguousarray(taps, dtype=np.float64)
    getattr(lib(), f"ox_apply_stencil_{_suffix(phi)}")(
        _ptr(phi), n, phi.shape[1], _ptr(t), float(scale), bc, _ptr(out), n)
    return out


def residual(phi, f, n, h, bc=BC_DIRICHLET0, want_r=True):
    """r = f - (1/h^2) S(phi); returns (r or None, max|r|, sum r^2)."""
    _check_phi(phi, n)
    _check_f(f, n)
    assert f.dtype == phi.dtype
    norms = np.zeros(2, dtype=np.float64)
    r = np.zeros((n, n), dtype=phi.dtype) if want_r else None
    getattr(lib(), f"ox_residual_{_suffix(phi)}")(
        _ptr(phi), n, phi.shape[1], _ptr(f), f.shape[1], float(h), bc,
        _ptr(r) if want_r else None, n, _ptr(norms))
    return r, float(norms[0]), float(norms[1])


def residual_terms(phi, f, n, h, bc=BC_DIRICHLET0):
    """The residual r = f - (1/h^2) S(phi) of every interior cell as the FP64 number
    whose square the norm adds (the arithmetic type's value, before rounding to
    storage); returns (rd (n x n float64), max|r|, sum r^2)."""
    _check_phi(phi, n)
    _check_f(f, n)
    assert f.dtype == phi.dtype
    norms = np.zeros(2, dtype=np.float64)
    rd = np.zeros((n, n), dtype=np.float64)
    getattr(lib(), f"ox_residual_terms_{_suffix(phi)}")(
        _ptr(phi), n, phi.shape[1], _ptr(f), f.shape[1], float(h), bc, _ptr(rd), _ptr(norms))
    return rd, float(norms[0]), float(norms[1])


def exact_sum_squares(rd: np.ndarray) -> float:
    """The sum of the FP64 squares rd*rd (each rounded once, as the norm forms them),
    added exactly and rounded once (math.fsum): the reference against which a sum of
    the same terms in any order is bounded by its own summation depth."""
    import math
    rd = np.asarray(rd, dtype=np.float64)
    return math.fsum((rd * rd).ravel().tolist())


def sweep(phi, f, n, h, lam, bc=BC_DIRICHLET0):
    """One sweep; returns (phi_out, max|r|, sum r^2) with the norms of the INPUT iterate."""
    _check_phi(phi, n)
    _check_f(f, n)
    out = np.zeros_like(phi)
    norms = np.zeros(2, dtype=np.float64)
    getattr(lib(), f"ox_sweep_{_suffix(phi)}")(
        _ptr(phi), _ptr(out), n, phi.shape[1], _ptr(f), f.shape[1], float(h), float(lam), bc,
        _ptr(norms))
    return out, float(norms[0]), float(norms[1])


def relax(phi, f, n, h, lam, nsweeps, bc=BC_DIRICHLET0, resmode=RES_FINAL, out=None):
    """nsweeps sweeps; returns (phi_out, max|r|, sum r^2).  Corners of out untouched."""
    _check_phi(phi, n)
    _check_f(f, n)
    assert f.dtype == phi.dtype
    if out is None:
        out = np.zeros_like(phi)
    norms = np.full(2, np.nan, dtype=np.float64)
    getattr(lib(), f"ox_relax_{_suffix(phi)}")(
        _ptr(phi), _ptr(out), n, phi.shape[1], _ptr(f), f.shape[1], float(h), float(lam),
        int(nsweeps), bc, resmode, _ptr(norms))
    return out, float(norms[0]), float(norms[1])


def relax_sides(phi, f, n, h, lam, nsweeps, bcs, resmode=RES_FINAL, out=None):
    """Like relax() with one boundary mode per side: bcs = (north, south, west, east).
    A GHOST_FIXED side holds its ghost layer as given (a box interface)."""
    _check_phi(phi, n)
    _check_f(f, n)
    assert f.dtype == phi.dtype and len(bcs) == 4
    if out is None:
        out = np.zeros_like(phi)
    b4 = np.ascontiguousarray(bcs, dtype=np.int32)
    norms = np.full(2, np.nan, dtype=np.float64)
    getattr(lib(), f"ox_relax_sides_{_suffix(phi)}")(
        _ptr(phi), _ptr(out), n, phi.shape[1], _ptr(f), f.shape[1], float(h), float(lam),
        int(nsweeps), _ptr(b4), resmode, _ptr(norms))
    return out, float(norms[0]), float(norms[1])


def exchange_boxes(phis, nbx, nby, n, bc=BC_DIRICHLET0):
    """Section IV's copy between the boxes of one domain, in place: every box's ghost ring
    (corners excepted) from its neighbours' adjacent interior rows and columns; on the
    domain's edge -(adjacent interior) for DIRICHLET0, the opposite edge's box for PERIODIC,
    unchanged for GHOST_FIXED.  phis: nbx * nby ghosted grids in box-row-major order (box
    b covers domain rows (b // nbx) * n .. and columns (b % nbx) * n ..)."""
    def neg(a):
        return a ^ np.uint16(0x8000) if a.dtype == np.uint16 else -a
    for b in range(nbx * nby):
        bi, bj = divmod(b, nbx)
        me = phis[b]
        for side, (di, dj) in enumerate(((-1, 0), (1, 0), (0, -1), (0, 1))):
            ni, nj = bi + di, bj + dj
            if not (0 <= ni < nby and 0 <= nj < nbx):
                if bc == BC_PERIODIC:
                    ni, nj = ni % nby, nj % nbx
                else:
                    if bc == BC_DIRICHLET0:
                        if side == 0:
                            me[0, 1:n + 1] = neg(me[1, 1:n + 1])
                        elif side == 1:
                            me[n + 1, 1:n + 1] = neg(me[n, 1:n + 1])
                        elif side == 2:
                            me[1:n + 1, 0] = neg(me[1:n + 1, 1])
                        else:
                            me[1:n + 1, n + 1] = neg(me[1:n + 1, n])
                    continue
            nb = phis[ni * nbx + nj]
            if side == 0:
                me[0, 1:n + 1] = nb[n, 1:n + 1]
            elif side == 1:
                me[n + 1, 1:n + 1] = nb[1, 1:n + 1]
            elif side == 2:
                me[1:n + 1, 0] = nb[1:n + 1, n]
            else:
                me[1:n + 1, n + 1] = nb[1:n + 1, 1]


def relax_boxes(phis, fs, nbx, nby, n, h, lam, nsweeps, exchange=1, bc=BC_DIRICHLET0):
    """A domain of boxes relaxed as the paper's Algorithm runs on Proto boxes: every
    `exchange` sweeps the ghost rings are exchanged (exchange_boxes), then every box
    relaxes `exchange` sweeps on its own with its ghost ring held (GHOST_FIXED).  Returns new
    grids (corners copied from the inputs)."""
    assert nsweeps % exchange == 0
    cur = [np.array(p, copy=True) for p in phis]
    for _ in range(nsweeps // exchange):
        exchange_boxes(cur, nbx, nby, n, bc)
        nxt = []
        for p, f in zip(cur, fs):
            out, _, _ = relax(p, f, n, h, lam, exchange, bc=BC_GHOST_FIXED, resmode=RES_NONE, out=p.copy())
            nxt.append(out)
        cur = nxt
    return cur


def refine(phi, f, n, h, lam, lowp, k_in, max_outer, rtol, bc=BC_DIRICHLET0):
    """FP64 iterative refinement around k_in low-precision sweeps (lowp 1=FP32, 2=BF16).

    phi (float64, ghosted) is updated in place; returns (outer_steps, max|r|, sum r^2)."""
    _check_phi(phi, n)
    _check_f(f, n)
    assert phi.dtype == np.float64 and f.dtype == np.float64
    norms = np.zeros(2, dtype=np.float64)
    k = lib().ox_refine(_ptr(phi), n, phi.shape[1], _ptr(f), f.shape[1], float(h), float(lam),
                        bc, int(lowp), int(k_in), int(max_outer), float(rtol), _ptr(norms))
    return int(k), float(norms[0]), float(norms[1])


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 bit patterns (RNE), element by element."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty(x.shape, dtype=np.uint16)
    lib().ox_f32_to_bf16_array(_ptr(x), _ptr(y), x.size)
    return y


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)
