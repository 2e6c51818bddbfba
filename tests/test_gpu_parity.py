"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: bit-exact for every element of phi (interior and edge ghosts) in FP64,
FP32 and BF16, and for max|r|; sum r^2 within gamma_D of the exact sum of the
oracle's own squares, D the GPU's summation depth (under 2e-13 relative at
these sizes; the two sides add the same squares in different orders)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_07931_amd as px
import workloads as W
from oracle import exact

import helpers as H

pytestmark = pytest.mark.gpu
OMEGA = 2.0 / 3.0


@pytest.fixture(scope="module")
def ctx():
    H.require_gpu()
    c = px.Context()
    yield c
    c.close()


def params(n, node_centred=False):
    h = 1.0 / (n + 1) if node_centred else 1.0 / n
    return h, OMEGA * h * h / 4.0


# --------------------------------------------------- manufactured 64 x 64 --

@pytest.mark.parametrize("tblock", range(1, 9))
def test_manufactured_64_fp64_matches_oracle_and_closed_form(ctx, tblock):
    n, N = 64, 100
    h, lam = params(n)
    f = W.manufactured_rhs(n)
    phi0 = np.zeros((n + 2, n + 2))
    print(f"case: manufactured n={n} sweeps={N} tblock={tblock}", flush=True)
    g, norms = H.gpu_relax(phi0, f, n, h, lam, N, "f64", ctx, tblock=tblock)
    ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, N, "f64")
    H.assert_grid_bitwise(g, ref, n)
    H.assert_norms(norms, mx, sq, n=n)
    cf = exact.manufactured_closed_form(n, N, OMEGA)
    assert norms[0] == pytest.approx(cf["res_max_final"], rel=1e-12)
    err = np.abs(g[1:n + 1, 1:n + 1] - W.manufactured_solution(n)).max()
    assert err == pytest.approx(cf["err_max"], rel=1e-12)


# ------------------------------------------------------- general parity --

CASES = [
    # dt, n, nsweeps, tblock, bc, resmode
    ("f64", 1, 3, 1, 0, 2), ("f64", 2, 5, 2, 0, 1), ("f64", 3, 7, 3, 1, 2),
    ("f64", 7, 9, 8, 0, 2), ("f64", 64, 13, 4, 0, 1), ("f64", 125, 11, 5, 0, 2),
    ("f64", 130, 16, 8, 1, 2), ("f64", 257, 9, 1, 0, 2), ("f64", 300, 12, 6, 1, 1),
    ("f64", 97, 0, 4, 0, 2), ("f64", 40, 17, 7, 0, 0),
    ("f32", 1, 4, 4, 0, 2), ("f32", 5, 6, 2, 1, 1), ("f32", 64, 10, 1, 0, 2),
    ("f32", 129, 12, 3, 0, 2), ("f32", 255, 16, 8, 1, 2), ("f32", 300, 9, 4, 0, 1),
    ("bf16", 3, 5, 5, 0, 2), ("bf16", 33, 8, 2, 1, 2), ("bf16", 130, 12, 4, 0, 1),
    ("bf16", 261, 16, 8, 0, 2),
    # one sweep per launch where a strip ends at column n: its right neighbour is the
    # ghost column, which must come from the boundary rule, not from memory
    ("f64", 255, 3, 1, 0, 2), ("f64", 383, 2, 1, 0, 0), ("f32", 511, 2, 1, 0, 2),
    # periodic (torus)
    ("f64", 1, 3, 1, 2, 2), ("f64", 7, 9, 8, 2, 2), ("f64", 64, 13, 4, 2, 1), ("f64", 255, 7, 1, 2, 2),
    ("f64", 300, 16, 8, 2, 2), ("f64", 130, 10, 5, 2, 0), ("f64", 97, 11, 2, 2, 2),
    ("f32", 129, 12, 3, 2, 2), ("f32", 300, 16, 8, 2, 1), ("f32", 511, 3, 1, 2, 2),
    ("bf16", 33, 8, 2, 2, 2), ("bf16", 261, 16, 8, 2, 2),
]


@pytest.mark.parametrize("dt,n,nsweeps,tblock,bc,resmode", CASES)
def test_relax_matches_oracle(ctx, dt, n, nsweeps, tblock, bc, resmode):
    h, lam = params(n)
    f = W.uniform_rhs(n, 1000 + n)
    phi0 = W.uniform_phi(n, 2000 + n)
    print(f"case: {dt} n={n} sweeps={nsweeps} tblock={tblock} bc={bc} res={resmode}", flush=True)
    g, norms = H.gpu_relax(phi0, f, n, h, lam, nsweeps, dt, ctx, tblock=tblock, bc=bc,
                           resmode=resmode)
    ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, nsweeps, dt, bc=bc, resmode=resmode)
    H.assert_grid_bitwise(g, ref, n)
    if bc == px.BC_PERIODIC and nsweeps > 0:  # on a torus the corners are written too
        for i, j in ((0, 0), (0, n + 1), (n + 1, 0), (n + 1, n + 1)):
            assert H.bits(g[i:i + 1, j]) == H.bits(ref[i:i + 1, j]), (i, j)
    if resmode != px.RES_NONE:
        H.assert_norms(norms, mx, sq, n=n)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_all_tblocks_and_tile_shapes_agree(ctx, dt):
    """k sweeps per launch and the tile height change nothing, bit for bit."""
    n, N = 203, 24
    h, lam = params(n)
    f = W.uniform_rhs(n, 5)
    phi0 = W.uniform_phi(n, 6)
    ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, N, dt)
    for rows in (0, 1, 3, 17, 300):
        ctx.set_tile_rows(rows)
        for tb in range(1, 9):
            print(f"case: {dt} rows={rows} tblock={tb}", flush=True)
            g, norms = H.gpu_relax(phi0, f, n, h, lam, N, dt, ctx, tblock=tb)
            H.assert_grid_bitwise(g, ref, n, what=f"rows={rows} tblock={tb}")
            H.assert_norms(norms, mx, sq, n=n)
    ctx.set_tile_rows(0)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_unaligned_layouts(ctx, dt):
    """ld = n+2 (rows not 16-byte aligned for FP32/BF16) and f packed n wide with no
    alignment help: the scalar paths give the same bits."""
    n, N = 131, 10
    h, lam = params(n)
    f = W.uniform_rhs(n, 7)
    phi0 = W.uniform_phi(n, 8)
    ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, N, dt)
    for ld, ld_f, fal in ((n + 2, n, False), (n + 3, n + 1, False), (None, None, True), (n + 2, None, True)):
        print(f"case: {dt} ld={ld} ld_f={ld_f} f_aligned={fal}", flush=True)
        g, norms = H.gpu_relax(phi0, f, n, h, lam, N, dt, ctx, tblock=3, ld=ld, ld_f=ld_f, f_aligned=fal)
        H.assert_grid_bitwise(g, ref, n, what=f"ld={ld} ld_f={ld_f}")
        H.assert_norms(norms, mx, sq, n=n)


def test_node_centred_ghost_fixed_closed_form(ctx):
    n, N = 64, 100
    h, lam = params(n, node_centred=True)
    f = -2 * np.pi ** 2 * W.sine_mode(n, 1, 1, node_centred=True)
    g, norms = H.gpu_relax(np.zeros((n + 2, n + 2)), f, n, h, lam, N, "f64", ctx, tblock=4, bc=1)
    cf = exact.manufactured_closed_form(n, N, OMEGA, node_centred=True)
    np.testing.assert_allclose(g[1:n + 1, 1:n + 1], cf["phi"], rtol=0, atol=5e-15)
    assert norms[0] == pytest.approx(cf["res_max_final"], rel=1e-12)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_autotuned_configuration_matches_oracle(dt):
    """The autotuner picks some (k, rows); relaxing with it (tblock = 0) changes no bit."""
    n, N = 300, 19
    h, lam = params(n)
    f = W.uniform_rhs(n, 31)
    phi0 = W.uniform_phi(n, 32)
    c = px.Context()
    pin = H.device_grid(phi0, n, dt)
    pout = torch.zeros_like(pin)
    fd = H.device_rhs(f, n, dt)
    k, rows, g = px.autotune(pin, pout, n, fd, c)
    assert 1 <= k <= 8 and 4 <= rows <= 128 and g > 0
    pout.fill_(H.SENTINEL)
    norms = torch.zeros(2, dtype=torch.float64, device="cuda")
    px.relax_fused(pin, pout, n, fd, h, lam, N, c, tblock=0, norms=norms)
    torch.cuda.synchronize()
    ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, N, dt)
    H.assert_grid_bitwise(H.to_storage_np(pout, dt), ref, n)
    H.assert_norms(norms.cpu().numpy(), mx, sq, n=n)
    c.close()


# ----------------------------------------------------- invariants on GPU --

def test_split_run_is_bitwise(ctx):
    n = 260
    h, lam = params(n)
    f = W.uniform_rhs(n, 9)
    phi0 = W.uniform_phi(n, 10)
    a, _ = H.gpu_relax(phi0, f, n, h, lam, 40, "f64", ctx, tblock=4)
    b, _ = H.gpu_relax(phi0, f, n, h, lam, 17, "f64", ctx, tblock=8)
    b, _ = H.gpu_relax(b[:, :n + 2], f, n, h, lam, 23, "f64", ctx, tblock=3)
    H.assert_grid_bitwise(a, b, n)


def test_lagged_equals_final_of_previous(ctx):
    n = 150
    h, lam = params(n)
    f = W.uniform_rhs(n, 11)
    phi0 = np.zeros((n + 2, n + 2))
    _, nl = H.gpu_relax(phi0, f, n, h, lam, 21, "f64", ctx, tblock=4, resmode=px.RES_LAGGED)
    _, nf = H.gpu_relax(phi0, f, n, h, lam, 20, "f64", ctx, tblock=4, resmode=px.RES_FINAL)
    assert nl[0] == nf[0]
    assert nl[1] == pytest.approx(nf[1], rel=1e-13)


def test_nan_in_rhs_propagates_to_max_norm(ctx):
    n = 70
    h, lam = params(n)
    f = W.uniform_rhs(n, 12)
    f[30, 40] = np.nan
    _, norms = H.gpu_relax(np.zeros((n + 2, n + 2)), f, n, h, lam, 6, "f64", ctx, tblock=2)
    assert np.isnan(norms[0]) and np.isnan(norms[1])


# ------------------------------------------ stencil / residual / unfused --

@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_apply_stencil_quadratic_exact(ctx, dt):
    n = 16 if dt == "bf16" else 200
    phi = W.quadratic_grid(n, 1, 0, 1, 0, 0, 0, shift=n // 2 + 1)
    pd = H.device_grid(phi, n, dt)
    out = torch.full((n, n + 5), 3.0, dtype=H.TORCH_DTYPE[dt], device="cuda")
    px.apply_stencil(pd, n, out, bc=px.BC_GHOST_FIXED)
    torch.cuda.synchronize()
    assert torch.all(out[:, :n].float() == 4.0)
    assert torch.all(out[:, n:].float() == 3.0)  # padding untouched


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("taps,scale,bc", [
    (px.LAPLACE_TAPS, 1.0, 0), (px.LAPLACE_TAPS, 4096.0, 1),
    ((1, 0, -1, 0, 0, 0, -1, 0, 1), 0.25, 0), ((0.5, 1, 0.25, 2, -3, 1, 0.125, -1, 0.75), 1.5, 0),
    ((0.5, 1, 0.25, 2, -3, 1, 0.125, -1, 0.75), 1.0, 1),
    (px.LAPLACE_TAPS, 1.0, 2), ((0.5, 1, 0.25, 2, -3, 1, 0.125, -1, 0.75), 1.0, 2),
])
def test_apply_stencil_matches_oracle(ctx, dt, taps, scale, bc):
    n = 77
    phi = W.uniform_phi(n, 13)
    pd = H.device_grid(phi, n, dt)
    out = torch.zeros((n, n), dtype=H.TORCH_DTYPE[dt], device="cuda")
    px.apply_stencil(pd, n, out, taps=taps, scale=scale, bc=bc)
    torch.cuda.synchronize()
    ref = oracle.apply_stencil(H.oracle_input(phi, dt), n, taps=taps, scale=scale, bc=bc)
    assert np.array_equal(H.bits(H.to_storage_np(out, dt)), H.bits(ref))


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("bc", [0, 1, 2])
def test_residual_matches_oracle(ctx, dt, bc):
    n = 123
    h, _ = params(n)
    phi = W.uniform_phi(n, 14)
    f = W.uniform_rhs(n, 15)
    pd = H.device_grid(phi, n, dt)
    fd = H.device_rhs(f, n, dt)
    r = torch.zeros((n, n), dtype=H.TORCH_DTYPE[dt], device="cuda")
    norms = torch.zeros(2, dtype=torch.float64, device="cuda")
    px.residual(pd, n, fd, h, norms, ctx, bc=bc, r=r)
    torch.cuda.synchronize()
    rr, mx, sq = H.oracle_residual_exact(phi, f, n, h, dt, bc=bc)
    assert np.array_equal(H.bits(H.to_storage_np(r, dt)), H.bits(rr))
    H.assert_norms(norms.cpu().numpy(), mx, sq, n=n)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_unfused_sweep_equals_fused(ctx, dt):
    """Proto-shaped sweep (stencil into a temporary, pointwise update in place, residual
    of the new iterate) gives the fused kernel's bits.  (In BF16 the temporary itself is
    stored in BF16, so the unfused form rounds once more by construction.)"""
    n, N = 190, 7
    h, lam = params(n)
    f = W.uniform_rhs(n, 16)
    phi0 = W.uniform_phi(n, 17)
    pd = H.device_grid(phi0, n, dt)
    fd = H.device_rhs(f, n, dt)
    tmp = torch.zeros((n, n), dtype=H.TORCH_DTYPE[dt], device="cuda")
    norms = torch.zeros(2, dtype=torch.float64, device="cuda")
    for _ in range(N):
        px.apply_stencil(pd, n, tmp)
        px.jacobi_update(pd, n, tmp, fd, h, lam)
    px.residual(pd, n, fd, h, norms, ctx)
    torch.cuda.synchronize()
    g, nf = H.gpu_relax(phi0, f, n, h, lam, N, dt, ctx, tblock=4)
    un = H.to_storage_np(pd, dt)
    inner = np.zeros((n + 2, n + 2), dtype=bool)
    inner[1:n + 1, 1:n + 1] = True  # the in-place update leaves ghosts alone
    H.assert_grid_bitwise(un, g, n, mask=inner)
    assert float(norms[0]) == nf[0]


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("k", [2, 5, 8])
def test_interior_unrolled_path_matches_oracle(dt, k):
    """Interior tiles of launches without norms with k + 1 a multiple of 3 run the
    unrolled-ring loop; several launches (the last one with final norms) at band heights
    that do and do not fill whole unrolled blocks give the oracle's result bit for bit.
    At n = 333 the 128-column FP64 waves get interior tiles in every direction; the
    256-column FP32 and BF16 waves get none below n of about 490 (their edge tiles are
    what this case checks), so their interior tiles are covered at n >= 520 in
    test_gpu_interior.py."""
    H.require_gpu()
    n = 333
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    phi0 = W.uniform_phi(n, 600 + k)
    f = W.uniform_rhs(n, 610 + k)
    ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, 3 * k + 1, dt)
    for rows in (8, 14, 29):
        c = px.Context()
        c.set_tile_rows(rows)
        print(f"case: {dt} k={k} rows={rows}", flush=True)
        got, nm = H.gpu_relax(phi0, f, n, h, lam, 3 * k + 1, dt, c, tblock=k)
        H.assert_grid_bitwise(got, ref, n, what=f"{dt} k={k} rows={rows}")
        H.assert_norms(nm, mx, sq, n=n)
        c.close()


def test_periodic_plain_solve_matches_oracle(ctx):
    """A torus with a zero-sum right-hand side: the plain solve converges, and its iterate
    is the oracle's after the same number of sweeps, bit for bit."""
    n = 48
    h, lam = params(n)
    f = W.uniform_rhs(n, 77)
    f -= f.mean()
    phi0 = np.zeros((n + 2, n + 2))
    pd = H.device_grid(phi0, n, "f64")
    fd = H.device_rhs(f, n, "f64")
    st = px.solve(pd, n, fd, h, lam, ctx, rtol=1e-6, check_every=256, bc=px.BC_PERIODIC)
    assert st.rel_res_max <= 1e-6 and st.sweeps % 256 == 0
    ref, _, _ = H.oracle_relax(phi0, f, n, h, lam, st.sweeps, "f64", bc=px.BC_PERIODIC)
    H.assert_grid_bitwise(H.to_storage_np(pd, "f64"), ref, n)


@pytest.mark.parametrize("dt,scale,resmode", [
    ("f64", 1e307, px.RES_NONE), ("f64", 1e-310, px.RES_FINAL),
    ("f32", 3e37, px.RES_NONE), ("f32", 1e-40, px.RES_FINAL)])
@pytest.mark.parametrize("k", [1, 8])
def test_extreme_magnitudes_bitwise(dt, scale, resmode, k):
    """Both ends of the floating-point range, interior and edge tiles: grids scaled so that the
    stencil sums reach about half the largest finite value (the kernel forms N - 4C as one
    fused multiply-add, which equals multiply-then-subtract while 4C stays finite; the
    residual, scaled by 1/h^2, overflows, so no norms there) and to subnormal magnitudes
    (gradual underflow on both sides)."""
    H.require_gpu()
    n = 333
    h, lam = params(n)
    phi0 = W.uniform_phi(n, 700 + k) * scale
    f = W.uniform_rhs(n, 710 + k) * scale
    sweeps = 2 * k + 1
    ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, sweeps, dt, resmode=resmode)
    c = px.Context()
    c.set_tile_rows(29)
    print(f"case: {dt} scale={scale:g} k={k} sweeps={sweeps}", flush=True)
    got, nm = H.gpu_relax(phi0, f, n, h, lam, sweeps, dt, c, tblock=k, resmode=resmode)
    c.close()
    H.assert_grid_bitwise(got, ref, n, what=f"{dt} scale={scale:g} k={k}")
    interior = np.abs(ref[1:n + 1, 1:n + 1])
    assert np.isfinite(interior).all() and interior.max() > 0.01 * scale
    if resmode != px.RES_NONE:
        H.assert_norms(nm, mx, sq, n=n)


# ------------------------------------------------------- band geometry --

def band_count(n, rows):
    return (n + 2 + rows - 1) // rows


# (n, rows): an odd band count (the last band streams down alone), an even one, 4-row bands
# (every band's pipeline drains before it has filled), a band meeting the next at the
# ghost row (n + 1 = 9 rows * 10: the last band holds only row n + 1), a one-band grid
GEOMETRY_GRIDS = [(100, 8), (100, 17), (61, 4), (89, 10), (30, 64), (777, 29)]


@pytest.mark.parametrize("k", [2, 5, 8])
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_band_geometry_edge_cases_match_oracle(dt, k):
    """The unrolled-ring loop (launches without norms, k + 1 a multiple of 3) on band
    layouts at the edges of its geometry, three launches (and, with a residual mode, a
    fourth on the generic loop), every boundary rule: bit for bit equal to the oracle."""
    H.require_gpu()
    assert band_count(100, 8) % 2 == 1 and band_count(100, 17) % 2 == 0
    assert (89 + 1) % 10 == 0 and band_count(30, 64) == 1
    for i, (n, rows) in enumerate(GEOMETRY_GRIDS):
        h, lam = params(n)
        bc = (0, 1, 2)[(i + k) % 3]
        rm = px.RES_NONE if i % 2 == 0 else px.RES_FINAL
        N = 3 * k + (0 if rm == px.RES_NONE else 1)
        phi0 = W.uniform_phi(n, 7300 + 10 * i + k)
        f = W.uniform_rhs(n, 7400 + 10 * i + k)
        c = px.Context()
        c.set_tile_rows(rows)
        print(f"case: geometry {dt} n={n} rows={rows} k={k} bc={bc} res={rm} sweeps={N}", flush=True)
        got, nm = H.gpu_relax(phi0, f, n, h, lam, N, dt, c, tblock=k, bc=bc, resmode=rm)
        c.close()
        ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, N, dt, bc=bc, resmode=rm)
        mask = np.ones((n + 2, n + 2), dtype=bool) if bc == px.BC_PERIODIC else None
        H.assert_grid_bitwise(got, ref, n, mask=mask, what=f"geometry {dt} n={n} rows={rows} k={k} bc={bc}")
        if rm != px.RES_NONE:
            H.assert_norms(nm, mx, sq, n=n, rows=rows)
