"""Shared helpers of the GPU tests: device buffers from numpy inputs, bitwise
comparison with the oracle, and the light-cone window check used at full size.

Inputs always come from ``workloads`` (seeded); the oracle gets them as numpy
arrays, the GPU as torch tensors converted by torch itself."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_2307_07931_amd as px

TORCH_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}
NP_DTYPE = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16}
SENTINEL = 7.0


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("these tests need a GPU (run with -m 'not gpu' on the CPU)")
    px.lib()


def oracle_input(x: np.ndarray, dt: str) -> np.ndarray:
    """float64 values -> the oracle's storage (float64, float32, or bf16 bits)."""
    if dt == "f64":
        return np.ascontiguousarray(x, dtype=np.float64)
    if dt == "f32":
        return np.ascontiguousarray(x, dtype=np.float32)
    return oracle.f32_to_bf16_bits(np.ascontiguousarray(x, dtype=np.float32))


def to_device_values(x: np.ndarray, dt: str) -> torch.Tensor:
    """float64 values -> device tensor of dtype dt, rounded by torch (FP64 -> FP32 -> BF16)."""
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")
    if dt == "f64":
        return t
    t = t.to(torch.float32)
    return t if dt == "f32" else t.to(torch.bfloat16)


def device_grid(x: np.ndarray, n: int, dt: str, ld: int | None = None) -> torch.Tensor:
    g = px.alloc_grid(n, TORCH_DTYPE[dt], ld=ld)
    g[:, :n + 2] = to_device_values(x, dt)
    return g


def device_rhs(f: np.ndarray, n: int, dt: str, ld_f: int | None = None, aligned: bool = True):
    if aligned:
        t = px.alloc_rhs(n, TORCH_DTYPE[dt], ld_f=ld_f)
    else:
        ld_f = ld_f or n
        t = torch.zeros((n, ld_f), dtype=TORCH_DTYPE[dt], device="cuda")
    t[:, :n] = to_device_values(f, dt)
    return t


def to_storage_np(t: torch.Tensor, dt: str) -> np.ndarray:
    """Device tensor -> numpy array in the oracle's storage representation."""
    c = t.detach().cpu()
    if dt == "bf16":
        return c.view(torch.int16).numpy().view(np.uint16).copy()
    return c.numpy().copy()


def bits(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a)
    return a.view({8: np.int64, 4: np.int32, 2: np.int16}[a.itemsize])


def noncorner_mask(n: int) -> np.ndarray:
    m = np.ones((n + 2, n + 2), dtype=bool)
    m[0, 0] = m[0, -1] = m[-1, 0] = m[-1, -1] = False
    return m


def assert_grid_bitwise(gpu: np.ndarray, ref: np.ndarray, n: int, mask: np.ndarray | None = None,
                        what: str = "phi"):
    g = bits(np.ascontiguousarray(gpu[:n + 2, :n + 2]))
    r = bits(np.ascontiguousarray(ref[:n + 2, :n + 2]))
    m = noncorner_mask(n) if mask is None else mask
    bad = (g != r) & m
    if bad.any():
        idx = np.argwhere(bad)
        i, j = idx[0]
        raise AssertionError(f"{what}: {bad.sum()} of {m.sum()} cells differ; first at ({i},{j}): "
                             f"gpu={gpu[i, j]!r} oracle={ref[i, j]!r}")


def gpu_relax(phi0: np.ndarray, f: np.ndarray, n: int, h: float, lam: float, nsweeps: int, dt: str,
              ctx, tblock: int = 0, bc: int = 0, resmode: int = px.RES_FINAL, ld=None, ld_f=None,
              f_aligned=True):
    """Runs px_relax_fused; returns (phi_out as storage numpy (n+2, ld), norms numpy[2])."""
    pin = device_grid(phi0, n, dt, ld=ld)
    pout = torch.full_like(pin, SENTINEL)
    fd = device_rhs(f, n, dt, ld_f=ld_f, aligned=f_aligned)
    norms = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    px.relax_fused(pin, pout, n, fd, h, lam, nsweeps, ctx, tblock=tblock, bc=bc, resmode=resmode,
                   norms=norms)
    torch.cuda.synchronize()
    return to_storage_np(pout, dt), norms.cpu().numpy()


def oracle_relax(phi0: np.ndarray, f: np.ndarray, n: int, h: float, lam: float, nsweeps: int,
                 dt: str, bc: int = 0, resmode: int = oracle.RES_FINAL, exact_sum: bool = True):
    """The oracle's nsweeps sweeps; returns (phi_out, max|r|, sum r^2).  With exact_sum
    the sum of squares returned is the exact sum (math.fsum) of the oracle's own FP64
    squares of the measured iterate (phi_out for FINAL, the iterate before the last sweep
    for LAGGED), after checking that the oracle's max is the max of those residuals and
    that its sequential row-major sum lies within its own bound of the exact one."""
    pin, fin = oracle_input(phi0, dt), oracle_input(f, dt)
    out, mx, sq = oracle.relax(pin, fin, n, h, lam, nsweeps, bc=bc, resmode=resmode)
    if not exact_sum or resmode == oracle.RES_NONE or (nsweeps == 0 and resmode == oracle.RES_LAGGED):
        return out, mx, sq
    if resmode == oracle.RES_FINAL:
        measured = out
    else:  # the norm of the last sweep's input: the iterate after nsweeps - 1 sweeps
        measured, _, _ = oracle.relax(pin, fin, n, h, lam, nsweeps - 1, bc=bc, resmode=oracle.RES_NONE)
    rd, mx2, sq2 = oracle.residual_terms(np.ascontiguousarray(measured), fin, n, h, bc=bc)
    if np.isnan(mx):
        assert np.isnan(mx2)
        return out, mx, sq
    assert mx2 == mx and sq2 == sq, (mx, mx2, sq, sq2)
    ex = oracle.exact_sum_squares(rd)
    # the oracle's own sum: n^2 - 1 additions in a row (recursive summation bound)
    assert abs(sq - ex) <= gamma(n * n) * ex + 1e-300, (sq, ex)
    return out, mx, ex


def oracle_residual_exact(phi: np.ndarray, f: np.ndarray, n: int, h: float, dt: str, bc: int = 0):
    """The oracle's residual of phi (storage of dt): (r in storage, max|r|, exact sum of
    the FP64 squares), the sum checked against the oracle's own sequential one."""
    pin, fin = oracle_input(phi, dt), oracle_input(f, dt)
    r, mx, sq = oracle.residual(pin, fin, n, h, bc=bc)
    rd, mx2, sq2 = oracle.residual_terms(pin, fin, n, h, bc=bc)
    assert (mx2, sq2) == (mx, sq) or np.isnan(mx)
    ex = oracle.exact_sum_squares(rd)
    assert np.isnan(mx) or abs(sq - ex) <= gamma(n * n) * ex + 1e-300, (sq, ex)
    return r, mx, ex


def gamma(depth: int) -> float:
    """gamma_d = d u / (1 - d u), u = 2^-53: a sum whose every term passes through at
    most d rounded additions differs from the exact sum by at most gamma_d times the sum
    of the magnitudes (Higham, Accuracy and Stability of Numerical Algorithms, Sec. 4.2)."""
    u = 2.0 ** -53
    return depth * u / (1.0 - depth * u)


def gpu_sum_depth(n: int, rows: int = 300) -> int:
    """Most additions any square passes through in the GPU's sum: a lane adds the cells
    of its band one after another (rows x 4 values at most), a wave combines its 64
    lanes in a 6-level tree, the partial of each wave (or 64-lane row segment, for the
    unfused kernels, plus 3 for their 4-wave blocks) is added sequentially by one of
    1024 threads, and those in a 10-level tree.  `rows`: the tallest band a launch of the
    test uses (300 is the tallest any test forces)."""
    per_lane = min(n + 2, rows) * 4
    partials = (n + 2) * ((n + 2 + 63) // 64)  # more than any launch writes
    return per_lane + 6 + 3 + (partials + 1023) // 1024 + 10


def assert_norms(gpu_norms, mx, sq, n=None, rel_sum=None, rows: int = 300):
    """max|r| bit for bit; the sum of squares within gamma_D of `sq`, where D is the
    GPU's summation depth (gpu_sum_depth) -- with `sq` the exact sum from oracle_relax
    that bounds the GPU's rounding alone, well under 1e-12 relative at every size tested."""
    gmx, gsq = float(gpu_norms[0]), float(gpu_norms[1])
    if np.isnan(mx):
        assert np.isnan(gmx)
        return
    assert gmx == mx, (gmx, mx)  # the max is exact
    tol = rel_sum if rel_sum is not None else (gamma(gpu_sum_depth(n, rows)) if n else 1e-12)
    assert tol <= 1e-12 or rel_sum is not None, tol
    assert abs(gsq - sq) <= tol * abs(sq) + 1e-300, (gsq, sq, tol)


def window_check(gpu_out: np.ndarray, phi0: np.ndarray, f: np.ndarray, n: int, h: float, lam: float,
                 nsweeps: int, r0: int, c0: int, W: int, dt: str) -> int:
    """Light-cone check of a full-size result: the oracle relaxes the W x W window whose
    top-left interior cell is (r0, c0), holding the window's interface ghosts fixed at
    their initial values (domain sides keep the Dirichlet reflection).  Window cells at
    least `nsweeps` cells from every fixed side are exact and must match bit for bit.
    Returns the number of cells compared."""
    assert 1 <= r0 and r0 + W - 1 <= n and 1 <= c0 and c0 + W - 1 <= n
    pw = np.ascontiguousarray(phi0[r0 - 1:r0 + W + 1, c0 - 1:c0 + W + 1])
    fw = np.ascontiguousarray(f[r0 - 1:r0 - 1 + W, c0 - 1:c0 - 1 + W])
    D, F = oracle.BC_DIRICHLET0, oracle.BC_GHOST_FIXED
    bcs = (D if r0 == 1 else F, D if r0 + W - 1 == n else F,
           D if c0 == 1 else F, D if c0 + W - 1 == n else F)
    out, _, _ = oracle.relax_sides(oracle_input(pw, dt), oracle_input(fw, dt), W, h, lam, nsweeps,
                                   bcs, resmode=oracle.RES_NONE)
    i = np.arange(W + 2)[:, None]
    j = np.arange(W + 2)[None, :]
    ok = np.ones((W + 2, W + 2), dtype=bool)
    # interior cells far enough from every fixed side
    ok &= (i >= 1) & (i <= W) & (j >= 1) & (j <= W)
    if bcs[0] == F:
        ok &= i >= nsweeps
    if bcs[1] == F:
        ok &= (W + 1 - i) >= nsweeps
    if bcs[2] == F:
        ok &= j >= nsweeps
    if bcs[3] == F:
        ok &= (W + 1 - j) >= nsweeps
    # Dirichlet ghost layers of valid cells are outputs too
    ghost = np.zeros_like(ok)
    if bcs[0] == D:
        ghost[0, 1:W + 1] = ok[1, 1:W + 1]
    if bcs[1] == D:
        ghost[W + 1, 1:W + 1] = ok[W, 1:W + 1]
    if bcs[2] == D:
        ghost[1:W + 1, 0] = ok[1:W + 1, 1]
    if bcs[3] == D:
        ghost[1:W + 1, W + 1] = ok[1:W + 1, W]
    mask = ok | ghost
    assert mask.sum() > 0
    gw = np.ascontiguousarray(gpu_out[r0 - 1:r0 + W + 1, c0 - 1:c0 + W + 1])
    assert_grid_bitwise(gw, out, W, mask=mask, what=f"window at ({r0},{c0})")
    return int(mask.sum())
