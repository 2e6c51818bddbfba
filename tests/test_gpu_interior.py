"""Interior tiles of the 256-column FP32 and BF16 waves against the oracle.

A tile is "interior" when every column it loads and every row it needs lie inside
[1, n]; such tiles take the loops without boundary substitution (and, for launches
without norms and k + 1 a multiple of 3, the unrolled-ring loop).  FP32 and BF16
waves hold 4 values per lane, 256 columns, so they get interior tiles only from
n of about 490 on; these cases run grids of 520, 777 and 1030 cells a side, every
k = 1..8 sweeps per launch, three boundary rules, three residual modes and band
heights that do and do not fill whole unrolled blocks -- the Jacobi step of
Section IV, Eq. 3 in the precisions of the mixed-precision and batched solvers.
Also here: batches with members of 512 to 1030 cells a side, and mixed-precision
solves at n = 520 (graph-replayed batch of one) and n = 1030 (host loop) with the
default inner sweep counts, against the oracle's refinement, bit for bit.

Bar: bit-exact phi (interior and ghost ring), max|r| bit for bit, sum r^2 within the
GPU's summation bound of the exact sum (helpers.assert_norms)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_07931_amd as px
import workloads as W

import helpers as H

pytestmark = pytest.mark.gpu
OMEGA = 2.0 / 3.0
SIZES = (520, 777, 1030)
# (bc, resmode) pairs; each (dtype, k) sees all nine over the three sizes
COMBOS = [(bc, rm) for bc in (px.BC_DIRICHLET0, px.BC_GHOST_FIXED, px.BC_PERIODIC)
          for rm in (px.RES_FINAL, px.RES_LAGGED, px.RES_NONE)]
ROWS = (8, 20, 29)


def params(n):
    h = 1.0 / n
    return h, OMEGA * h * h / 4.0


def interior_tiles(V: int, n: int, levels: int, rows: int) -> int:
    """Tiles of a launch that load only interior columns and need only interior rows
    (the same partition the library uses: waves of 64 V columns recomputing a halo of
    `levels` columns rounded to V on each side; one level: disjoint strips that also
    read the column right of the strip)."""
    halo = 0 if levels == 1 else (levels + V - 1) // V * V
    stride = 64 * V - 2 * halo
    tiles_x = (n + 2 + stride - 1) // stride
    tiles_y = (n + 2 + rows - 1) // rows
    count = 0
    for ty in range(tiles_y):
        y0, y1 = ty * rows, min(ty * rows + rows, n + 2)
        if not (y0 - levels >= 1 and y1 + levels - 1 <= n):
            continue
        for tx in range(tiles_x):
            c0 = tx * stride - halo
            if c0 >= 1 and c0 + 64 * V - (0 if levels == 1 else 1) <= n:
                count += 1
    return count


@pytest.mark.parametrize("k", range(1, 9))
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_low_precision_interior_tiles_match_oracle(dt, n, k):
    H.require_gpu()
    h, lam = params(n)
    phi0 = W.uniform_phi(n, 3000 + 10 * k + n % 7)
    f = W.uniform_rhs(n, 3100 + 10 * k + n % 7)
    N = 3 * k  # three launches of k sweeps; the last one takes the residual mode
    ni = SIZES.index(n)
    for i, rows in enumerate(ROWS):
        bc, rm = COMBOS[(3 * ni + i + k) % 9]
        levels = k + (1 if rm == px.RES_FINAL else 0)
        assert interior_tiles(4, n, k, rows) > 0 and interior_tiles(4, n, levels, rows) > 0
        c = px.Context()
        c.set_tile_rows(rows)
        print(f"case: {dt} n={n} k={k} rows={rows} bc={bc} res={rm} sweeps={N}", flush=True)
        got, nm = H.gpu_relax(phi0, f, n, h, lam, N, dt, c, tblock=k, bc=bc, resmode=rm)
        c.close()
        ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, N, dt, bc=bc, resmode=rm)
        H.assert_grid_bitwise(got, ref, n, what=f"{dt} n={n} k={k} rows={rows} bc={bc} res={rm}")
        if bc == px.BC_PERIODIC:
            for a, b in ((0, 0), (0, n + 1), (n + 1, 0), (n + 1, n + 1)):
                assert H.bits(got[a:a + 1, b]) == H.bits(ref[a:a + 1, b]), (a, b)
        if rm != px.RES_NONE:
            H.assert_norms(nm, mx, sq, n=n, rows=rows)


@pytest.mark.parametrize("k", [1, 4, 5, 8])
def test_fp64_interior_tiles_at_bench_band_height(k):
    """FP64 at n = 1030 with the 47-row bands the 4096^2 benchmark tunes to."""
    H.require_gpu()
    n = 1030
    h, lam = params(n)
    phi0 = W.uniform_phi(n, 3200 + k)
    f = W.uniform_rhs(n, 3300 + k)
    N = 3 * k + 1
    assert interior_tiles(2, n, k, 47) > 0
    c = px.Context()
    c.set_tile_rows(47)
    print(f"case: f64 n={n} k={k} rows=47 sweeps={N}", flush=True)
    got, nm = H.gpu_relax(phi0, f, n, h, lam, N, "f64", c, tblock=k)
    c.close()
    ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, N, "f64")
    H.assert_grid_bitwise(got, ref, n, what=f"f64 n={n} k={k}")
    H.assert_norms(nm, mx, sq, n=n, rows=47)


BATCH_SIZES = [512, 1030, 64, 777, 520, 129]


@pytest.mark.parametrize("dt,tblock,nsweeps", [("f32", 8, 19), ("bf16", 5, 13), ("f32", 1, 3), ("bf16", 8, 16),
                                               ("f32", 2, 7)])
def test_batched_large_members_match_oracle(dt, tblock, nsweeps):
    """Batch members of 512 to 1030 cells a side (interior tiles of 256-column waves) in
    one persistent launch per k sweeps, each equal to the oracle bit for bit."""
    H.require_gpu()
    c = px.Context()
    items, refs = [], []
    for j, n in enumerate(BATCH_SIZES):
        h, lam = params(n)
        phi0 = W.uniform_phi(n, 3400 + j)
        f = W.uniform_rhs(n, 3500 + j)
        items.append((H.device_grid(phi0, n, dt), H.device_rhs(f, n, dt), n, h, lam))
        refs.append((phi0, f, n, h, lam))
    norms = torch.full((2 * len(items),), float("nan"), dtype=torch.float64, device="cuda")
    print(f"case: batch {dt} tblock={tblock} sweeps={nsweeps} sizes={BATCH_SIZES}", flush=True)
    px.relax_batched(items, nsweeps, c, tblock=tblock, norms=norms)
    torch.cuda.synchronize()
    nm = norms.cpu().numpy()
    for j, ((phi, _, n, _, _), (phi0, f, _, h, lam)) in enumerate(zip(items, refs)):
        ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, nsweeps, dt)
        H.assert_grid_bitwise(H.to_storage_np(phi, dt), ref, n, what=f"member {j} (n={n})")
        H.assert_norms(nm[2 * j:2 * j + 2], mx, sq, n=n)
    c.close()


@pytest.mark.parametrize("n,mode,lowp,inner,steps", [
    (520, px.SOLVE_MIXED_F32, 1, 1024, 3), (520, px.SOLVE_MIXED_BF16, 2, 128, 6),
    (1030, px.SOLVE_MIXED_F32, 1, 1024, 2), (1030, px.SOLVE_MIXED_BF16, 2, 128, 4)])
def test_mixed_solve_default_inner_matches_oracle_refinement(n, mode, lowp, inner, steps):
    """Mixed-precision solves with the default inner sweep counts (1024 FP32, 128 BF16 per
    FP64 step), stopped by the sweep budget after `steps` outer steps, equal the oracle's
    refinement after the same steps bit for bit (phi and max|r|).  n = 520 runs as a
    graph-replayed batch of one, n = 1030 as the host-driven loop."""
    H.require_gpu()
    h, lam = params(n)
    f = W.grf_rhs(n, 3600 + n + lowp)
    c = px.Context()
    phi = H.device_grid(np.zeros((n + 2, n + 2)), n, "f64")
    fd = H.device_rhs(f, n, "f64")
    print(f"case: mixed lowp={lowp} n={n} inner=default({inner}) steps={steps}", flush=True)
    st = px.solve(phi, n, fd, h, lam, c, mode=mode, rtol=1e-14, max_sweeps=steps * inner,
                  raise_on_error=False)
    c.close()
    assert st.status == px.ENOTCONV and st.sweeps == steps * inner and st.outer_steps == steps, st
    ref = np.zeros((n + 2, n + 2))
    k, mx, _ = oracle.refine(ref, f, n, h, lam, lowp, inner, steps, 1e-14)
    assert k == steps
    inner_mask = np.zeros((n + 2, n + 2), dtype=bool)
    inner_mask[1:n + 1, 1:n + 1] = True
    H.assert_grid_bitwise(H.to_storage_np(phi, "f64"), ref, n, mask=inner_mask, what=f"mixed n={n} lowp={lowp}")
    assert st.res_max == mx, (st.res_max, mx)
