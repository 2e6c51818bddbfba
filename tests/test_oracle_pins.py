"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here retypes the oracle's sweep: each check compares the oracle with
an independent fact -- an exact polynomial identity, the eigen-structure of
the discrete Laplacian (closed forms), a dense brute-force matrix iteration,
an exact DST solve, the index map printed in the paper, or a library
rounding routine.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
OMEGA = 2.0 / 3.0


def lam_of(n, omega=OMEGA, node_centred=False):
    h = 1.0 / (n + 1) if node_centred else 1.0 / n
    return h, omega * h * h / 4.0


# ---------------------------------------------------------------- stencil --

@pytest.mark.parametrize("coef", [(1, 0, 0, 0, 0, 0), (0, 0, 1, 0, 0, 0), (3, 5, -2, 7, -11, 13),
                                  (-4, 9, 6, 1, 2, 3), (2, -3, 2, 0, 0, -100)])
@pytest.mark.parametrize("n", [5, 16, 33])
def test_laplacian_of_quadratic_is_exact_f64(coef, n):
    """The 5-point stencil of a quadratic a i^2 + b ij + c j^2 + ... is 2(a + c), exactly."""
    a, b, c, d, e, g = coef
    phi = W.quadratic_grid(n, a, b, c, d, e, g)
    out = oracle.apply_stencil(phi, n, bc=oracle.BC_GHOST_FIXED)
    assert np.all(out == 2.0 * (a + c))


def test_laplacian_of_quadratic_is_exact_f32():
    n = 1024  # values up to 2*512^2, every intermediate below 2^24
    phi = W.quadratic_grid(n, 1, 0, 1, 0, 0, 0, shift=n // 2 + 1).astype(np.float32)
    out = oracle.apply_stencil(phi, n, bc=oracle.BC_GHOST_FIXED)
    assert out.dtype == np.float32 and np.all(out == np.float32(4.0))


def test_laplacian_of_quadratic_is_exact_bf16():
    n = 16  # integers below 256 are exact in bfloat16
    phi = W.quadratic_grid(n, 1, 0, 1, 0, 0, 0, shift=n // 2 + 1)
    assert phi.max() < 256
    bits = oracle.f32_to_bf16_bits(phi.astype(np.float32))
    out = oracle.apply_stencil(bits, n, bc=oracle.BC_GHOST_FIXED)
    assert np.all(oracle.bf16_bits_to_f32(out) == 4.0)


def test_general_taps_cross_derivative_of_quadratic():
    """Taps [1,0,-1; 0,0,0; -1,0,1]/4 give the mixed derivative: on b*ij it is exactly b."""
    n = 12
    taps = (1, 0, -1, 0, 0, 0, -1, 0, 1)
    phi = W.quadratic_grid(n, 2, 6, -1, 3, 4, 5)
    out = oracle.apply_stencil(phi, n, taps=taps, scale=0.25, bc=oracle.BC_GHOST_FIXED)
    assert np.all(out == 6.0)


def test_stencil_matches_paper_index_map_and_order():
    """Fig. 5's index map and evaluation order on a 64x64 box stored 66 wide: the oracle's
    Laplacian at interior point i equals ((((X[b+1]-4X[b+67])+X[b+66])+X[b+68])+X[b+133])
    bit for bit (pins the layout orientation and the association of the sum)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_index_map.json")))
    n, m, c0 = g["n"], g["m"], g["centre_offset"]
    assert g["rho_offset_in_concatenated_input"] == m * m
    assert np.array_equal(np.array(g["filter_taps_rowwise"], dtype=float).ravel(),
                          np.array(oracle.LAPLACE_TAPS))
    X = W.rng(11).uniform(-1, 1, size=m * m)
    out = oracle.apply_stencil(X.reshape(m, m).copy(), n, bc=oracle.BC_GHOST_FIXED)
    o1, o2, o3, o4 = g["neighbour_offsets_in_sum_order"]
    for i, b in g["samples_i_to_b"]:
        assert b == m * (i // n) + i % n
    for i in range(n * n):
        b = m * (i // n) + i % n
        s = (((X[b + o1] + g["centre_coefficient"] * X[b + c0]) + X[b + o2]) + X[b + o3]) + X[b + o4]
        assert out.ravel()[i] == s
    # and the centre of point i is padded cell (i//n + 1, i%n + 1)
    assert all((m * (i // n + 1) + (i % n + 1)) == m * (i // n) + i % n + c0 for i in range(n * n))


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("bc", [oracle.BC_DIRICHLET0, oracle.BC_GHOST_FIXED, oracle.BC_PERIODIC])
def test_residual_and_sweep_use_the_pinned_stencil(dt, bc):
    """The Laplacian pass behind every residual and sweep is the generic stencil pass of
    the test above (pinned to Fig. 5's index map and order), bit for bit: the residual is
    r = f - c S(phi) and the sweep is phi' = (phi + w S(phi)) - lambda f with S from
    apply_stencil, each operation rounded on its own in the storage precision."""
    n = 37
    h, lam = lam_of(n)
    phi = W.rng(21).uniform(-1, 1, size=(n + 2, n + 2)).astype(dt)
    f = W.rng(22).uniform(-1, 1, size=(n, n)).astype(dt)
    S = oracle.apply_stencil(phi, n, bc=bc)
    c = dt(1.0 / (h * h))
    w = dt(lam / (h * h))
    r, _, _ = oracle.residual(phi, f, n, h, bc=bc)
    assert np.array_equal(r.view(np.uint8), (f - c * S).view(np.uint8))
    out, _, _ = oracle.sweep(phi, f, n, h, lam, bc=bc)
    C = phi[1:n + 1, 1:n + 1]
    upd = (C + w * S) - dt(lam) * f
    assert np.array_equal(out[1:n + 1, 1:n + 1].view(np.uint8), upd.view(np.uint8))


def test_threads_do_not_change_results():
    """The oracle's row loops run on several threads; every output, the sum of squares
    included, is the same bit for bit at any thread count."""
    n, N = 131, 9
    h, lam = lam_of(n)
    f = W.uniform_rhs(n, 23)
    phi0 = W.uniform_phi(n, 24)
    keep = oracle.get_threads()
    try:
        res = []
        for t in (1, 3, 8):
            oracle.set_threads(t)
            res.append(oracle.relax(phi0, f, n, h, lam, N))
        for out, mx, sq in res[1:]:
            assert np.array_equal(out.view(np.int64), res[0][0].view(np.int64))
            assert (mx, sq) == (res[0][1], res[0][2])
    finally:
        oracle.set_threads(keep)


# ------------------------------------------------------ eigen-structure --

@pytest.mark.parametrize("p,q", [(1, 1), (2, 3), (7, 1), (16, 16), (31, 5), (32, 32)])
def test_per_mode_damping_cell_centred(p, q):
    """With f = 0 a sine mode is damped by exactly g_pq per sweep."""
    n, N = 32, 40
    h, lam = lam_of(n)
    mode = W.sine_mode(n, p, q)
    phi0 = W.embed(mode, n, n + 2)
    out, _, _ = oracle.relax(phi0, np.zeros((n, n)), n, h, lam, N, resmode=oracle.RES_NONE)
    g = exact.mode_factor(n, p, q, OMEGA)
    np.testing.assert_allclose(out[1:-1, 1:-1], g ** N * mode, rtol=0, atol=2e-14)
    # odd-reflection ghosts on output
    assert np.array_equal(out[0, 1:-1], -out[1, 1:-1])
    assert np.array_equal(out[1:-1, -1], -out[1:-1, -2])


@pytest.mark.parametrize("p,q", [(1, 1), (3, 8), (20, 20)])
def test_per_mode_damping_node_centred(p, q):
    """Node-centred variant: zero ghosts held fixed, h = 1/(n+1)."""
    n, N = 20, 30
    h, lam = lam_of(n, node_centred=True)
    mode = W.sine_mode(n, p, q, node_centred=True)
    out, _, _ = oracle.relax(W.embed(mode, n, n + 4), np.zeros((n, n)), n, h, lam, N,
                             bc=oracle.BC_GHOST_FIXED, resmode=oracle.RES_NONE)
    g = exact.mode_factor(n, p, q, OMEGA, node_centred=True)
    np.testing.assert_allclose(out[1:-1, 1:n + 1], g ** N * mode, rtol=0, atol=2e-14)
    assert np.all(out[0, 1:n + 1] == 0) and np.all(out[1:-1, 0] == 0)


def test_top_mode_factor_is_one_minus_two_omega():
    """The (n, n) mode is damped by 1 - 2 omega (sin^2(pi/2) = 1): -1/3 at omega = 2/3."""
    assert exact.mode_factor(64, 64, 64, OMEGA) == pytest.approx(-1.0 / 3.0, abs=1e-15)


# -------------------------------------------------- manufactured problem --

def test_manufactured_64_closed_form():
    """64x64, f = -2 pi^2 sin sin at cell centres, phi0 = 0, 100 sweeps, omega = 2/3:
    sin(pi x) sin(pi y) is the (1,1) eigenmode, so every quantity has a closed form."""
    n, N = 64, 100
    h, lam = lam_of(n)
    cf = exact.manufactured_closed_form(n, N, OMEGA)
    assert cf["lambda"] == lam and cf["w"] == pytest.approx(1.0 / 6.0, rel=1e-15)
    f = W.manufactured_rhs(n)
    out, mx, sq = oracle.relax(np.zeros((n + 2, n + 2)), f, n, h, lam, N)
    np.testing.assert_allclose(out[1:-1, 1:-1], cf["phi"], rtol=0, atol=5e-15)
    assert mx == pytest.approx(cf["res_max_final"], rel=1e-12)
    assert sq == pytest.approx(cf["res_l2sq_final"], rel=1e-12)
    _, mxl, _ = oracle.relax(np.zeros((n + 2, n + 2)), f, n, h, lam, N, resmode=oracle.RES_LAGGED)
    assert mxl == pytest.approx(cf["res_max_lagged"], rel=1e-12)
    err = np.abs(out[1:-1, 1:-1] - W.manufactured_solution(n))
    assert err.max() == pytest.approx(cf["err_max"], rel=1e-12)
    assert np.sqrt(np.mean(err ** 2)) == pytest.approx(cf["err_rms"], rel=1e-12)
    # the numbers themselves (rel. residual g^100, the FP64 values quoted in the docs)
    assert cf["rel_res"] == pytest.approx(0.922806988355026, rel=1e-13)
    assert mx == pytest.approx(18.2045091556517, rel=1e-12)


def test_manufactured_node_centred_closed_form():
    n, N = 64, 100
    h, lam = lam_of(n, node_centred=True)
    cf = exact.manufactured_closed_form(n, N, OMEGA, node_centred=True)
    f = -2 * np.pi ** 2 * W.sine_mode(n, 1, 1, node_centred=True)
    out, mx, _ = oracle.relax(np.zeros((n + 2, n + 2)), f, n, h, lam, N, bc=oracle.BC_GHOST_FIXED)
    np.testing.assert_allclose(out[1:-1, 1:-1], cf["phi"], rtol=0, atol=5e-15)
    assert mx == pytest.approx(cf["res_max_final"], rel=1e-12)


def test_second_order_convergence_of_discrete_solution():
    """The exact discrete solution converges to sin sin at second order (ratios -> 4),
    with the closed-form error |s - 1| max|u|."""
    errs = []
    for n in (16, 32, 64, 128, 256):
        phi_h = exact.dst_solve(W.manufactured_rhs(n), 1.0 / n)
        e = np.abs(phi_h - W.manufactured_solution(n)).max()
        assert e == pytest.approx(exact.manufactured_closed_form(n, 1, OMEGA)["disc_err_max"], rel=1e-9)
        errs.append(e)
    ratios = [errs[k] / errs[k + 1] for k in range(len(errs) - 1)]
    assert all(3.9 < r < 4.01 for r in ratios), ratios
    assert ratios[-1] == pytest.approx(4.0, abs=2e-3)


# ----------------------------------------------------------- brute force --

@pytest.mark.parametrize("n", [4, 8, 12])
def test_dst_solve_matches_dense_solve(n):
    f = W.uniform_rhs(n, 100 + n)
    h = 1.0 / n
    a = exact.dst_solve(f, h)
    b = exact.dense_solve(f, h)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("node_centred", [False, True])
def test_sweeps_match_dense_matrix_iteration(node_centred):
    n, N = 8, 25
    h, lam = lam_of(n, node_centred=node_centred)
    f = W.uniform_rhs(n, 7)
    phi0 = W.uniform_phi(n, 8)
    bc = oracle.BC_GHOST_FIXED if node_centred else oracle.BC_DIRICHLET0
    if node_centred:
        phi0[0, :] = phi0[-1, :] = phi0[:, 0] = phi0[:, -1] = 0.0
    out, mx, sq = oracle.relax(phi0, f, n, h, lam, N, bc=bc)
    ref = exact.dense_jacobi(phi0[1:-1, 1:-1], f, h, lam, N, node_centred=node_centred)
    assert np.abs(out[1:-1, 1:-1] - ref).max() <= 1e-13 * np.abs(ref).max()
    A = exact.dense_laplacian(n, h, node_centred)
    r = f.ravel() - A @ ref.ravel()
    assert mx == pytest.approx(np.abs(r).max(), rel=1e-10)
    assert sq == pytest.approx(np.sum(r * r), rel=1e-10)


def test_residual_matches_dense_product():
    n = 10
    h = 1.0 / n
    phi = W.uniform_phi(n, 3)
    f = W.uniform_rhs(n, 4)
    r, mx, sq = oracle.residual(phi, f, n, h)
    ref = f.ravel() - exact.dense_laplacian(n, h) @ phi[1:-1, 1:-1].ravel()
    assert np.abs(r.ravel() - ref).max() <= 1e-13 * np.abs(ref).max()
    assert mx == np.abs(r).max()


def test_exact_solution_is_a_fixed_point():
    n = 64
    h, lam = lam_of(n)
    f = W.grf_rhs(n, 21)
    phi = W.embed(exact.dst_solve(f, h), n, n + 2)
    _, mx, _ = oracle.residual(phi, f, n, h)
    assert mx <= 1e-11 * np.abs(f).max()
    out, _, _ = oracle.relax(phi, f, n, h, lam, 5, resmode=oracle.RES_NONE)
    assert np.abs(out[1:-1, 1:-1] - phi[1:-1, 1:-1]).max() <= 1e-13 * np.abs(phi).max()


def test_residual_of_zero_is_rhs():
    n = 16
    f = W.uniform_rhs(n, 5)
    r, mx, _ = oracle.residual(np.zeros((n + 2, n + 2)), f, n, 1.0 / n)
    assert np.array_equal(r, f) and mx == np.abs(f).max()


# ------------------------------------------------------------ invariants --

def test_lagged_norm_is_final_norm_of_previous_iterate():
    n = 24
    h, lam = lam_of(n)
    f = W.uniform_rhs(n, 9)
    phi0 = np.zeros((n + 2, n + 2))
    _, mxl, sql = oracle.relax(phi0, f, n, h, lam, 17, resmode=oracle.RES_LAGGED)
    _, mxf, sqf = oracle.relax(phi0, f, n, h, lam, 16, resmode=oracle.RES_FINAL)
    assert mxl == mxf and sql == sqf


def test_split_run_is_bitwise():
    n = 20
    h, lam = lam_of(n)
    f = W.uniform_rhs(n, 10)
    phi0 = W.embed(W.uniform_rhs(n, 11), n, n + 2)
    a, _, _ = oracle.relax(phi0, f, n, h, lam, 30)
    b, _, _ = oracle.relax(phi0, f, n, h, lam, 13)
    b, _, _ = oracle.relax(b, f, n, h, lam, 17)
    assert np.array_equal(a[1:-1], b[1:-1])


def test_nan_propagates_into_max_norm():
    n = 8
    f = W.uniform_rhs(n, 12)
    f[3, 4] = np.nan
    _, mx, sq = oracle.residual(np.zeros((n + 2, n + 2)), f, n, 1.0 / n)
    assert np.isnan(mx) and np.isnan(sq)


# ---------------------------------------------------- reduced precision --

def test_bf16_rounding_matches_library_rne():
    torch = pytest.importorskip("torch")
    x = np.concatenate([
        W.rng(1).standard_normal(200000).astype(np.float32) * np.float32(1e3),
        np.array([0.0, -0.0, 1.0, np.inf, -np.inf, 3.0e38, 1e-40, -1e-42], dtype=np.float32),
        # exact ties between two bfloat16 neighbours, both parities
        (np.arange(1, 2000, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
    ])
    ours = oracle.f32_to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    nan = oracle.f32_to_bf16_bits(np.array([np.nan], dtype=np.float32))
    assert np.isnan(oracle.bf16_bits_to_f32(nan))[0]


def test_f32_variant_closed_form():
    n, N = 64, 100
    h, lam = lam_of(n)
    cf = exact.manufactured_closed_form(n, N, OMEGA)
    f = W.manufactured_rhs(n).astype(np.float32)
    out, mx, _ = oracle.relax(np.zeros((n + 2, n + 2), np.float32), f, n, h, lam, N)
    np.testing.assert_allclose(out[1:-1, 1:-1], cf["phi"], rtol=0, atol=2e-5)
    assert mx == pytest.approx(cf["res_max_final"], rel=2e-3)


def test_bf16_variant_damps_modes():
    n, N = 32, 10
    h, lam = lam_of(n)
    mode = W.sine_mode(n, 3, 2)
    bits = oracle.f32_to_bf16_bits(W.embed(mode, n, n + 2).astype(np.float32))
    fz = np.zeros((n, n), np.uint16)
    out, _, _ = oracle.relax(bits, fz, n, h, lam, N, resmode=oracle.RES_NONE)
    g = exact.mode_factor(n, 3, 2, OMEGA)
    np.testing.assert_allclose(oracle.bf16_bits_to_f32(out)[1:-1, 1:-1], g ** N * mode, atol=N * 2 ** -8)


@pytest.mark.parametrize("lowp,k_in", [(1, 64), (2, 8), (2, 32)])
def test_refinement_reaches_fp64_accuracy(lowp, k_in):
    """Low-precision inner sweeps with FP64 refinement reach an FP64-level residual and the
    DST-exact solution; the outer step count follows the FP64 per-sweep rate."""
    n = 32
    h, lam = lam_of(n)
    f = W.grf_rhs(n, 31)
    phi = np.zeros((n + 2, n + 2))
    steps, mx, _ = oracle.refine(phi, f, n, h, lam, lowp, k_in, 20000, 1e-12)
    assert mx <= 1e-12 * np.abs(f).max()
    ex = exact.dst_solve(f, h)
    assert np.abs(phi[1:-1, 1:-1] - ex).max() <= 1e-11 * np.abs(ex).max()
    # plain FP64 Jacobi needs about log(1e-12)/log(g_11) sweeps; refinement must not need
    # many more (the inner solves restart, so the rate per sweep is at most the FP64 rate)
    g = exact.mode_factor(n, 1, 1, OMEGA)
    plain = np.log(1e-12) / np.log(g)
    assert steps * k_in <= 1.25 * plain + 2 * k_in, (steps * k_in, plain)


# ------------------------------------------------- box interfaces (windows) --

def test_window_with_fixed_interface_ghosts_matches_full_grid():
    """A sub-box whose interface ghost layers are held at their initial values reproduces
    the full-grid sweeps exactly on every cell at least N cells from those interfaces
    (information travels one cell per sweep), and not one cell closer."""
    import helpers
    n, N, B = 48, 9, 30
    h, lam = lam_of(n)
    f = W.uniform_rhs(n, 41)
    phi0 = W.uniform_phi(n, 42)
    full, _, _ = oracle.relax(phi0, f, n, h, lam, N, resmode=oracle.RES_NONE)
    for r0, c0 in ((1, 1), (n - B + 1, 1), (10, 12), (n - B + 1, n - B + 1)):
        assert helpers.window_check(full, phi0, f, n, h, lam, N, r0, c0, B, "f64") > 0
    # one row closer to a fixed interface the window result is no longer exact
    pw = np.ascontiguousarray(phi0[9:9 + B + 2, 11:11 + B + 2])
    fw = np.ascontiguousarray(f[9:9 + B, 11:11 + B])
    F = oracle.BC_GHOST_FIXED
    out, _, _ = oracle.relax_sides(pw, fw, B, h, lam, N, (F, F, F, F), resmode=oracle.RES_NONE)
    assert np.any(out[N - 1, N:B + 2 - N] != full[9 + N - 1, 11 + N:11 + B + 2 - N])


# ------------------------------------------------------ periodic variant --
# On a torus (Proto's own boundary) the discrete Fourier modes are the eigenvectors of
# the 5-point stencil: S cos(2 pi (p i + q j) / n) = -4 (sin^2(pi p / n) + sin^2(pi q / n))
# times the mode, so with f = 0 one sweep multiplies the mode by
# g = 1 - omega (sin^2(pi p / n) + sin^2(pi q / n)).

def periodic_mode(n, p, q):
    i = np.arange(1, n + 1)[:, None]
    j = np.arange(1, n + 1)[None, :]
    return np.cos(2 * np.pi * (p * i + q * j) / n + 0.3)


def torus_laplacian(n, h):
    """Dense periodic 5-point Laplacian (circulant), written out cell by cell."""
    A = np.zeros((n * n, n * n))
    for i in range(n):
        for j in range(n):
            k = i * n + j
            A[k, k] -= 4.0
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                A[k, ((i + di) % n) * n + (j + dj) % n] += 1.0
    return A / (h * h)


@pytest.mark.parametrize("p,q", [(0, 1), (1, 1), (2, 5), (8, 0), (8, 8), (3, 13)])
def test_periodic_mode_damping(p, q):
    n, N = 16, 30
    h, lam = lam_of(n)
    mode = periodic_mode(n, p, q)
    out, _, _ = oracle.relax(W.embed(mode, n, n + 2), np.zeros((n, n)), n, h, lam, N,
                             bc=oracle.BC_PERIODIC, resmode=oracle.RES_NONE)
    g = 1.0 - OMEGA * (np.sin(np.pi * p / n) ** 2 + np.sin(np.pi * q / n) ** 2)
    np.testing.assert_allclose(out[1:-1, 1:-1], g ** N * mode, rtol=0, atol=2e-14)
    # ghosts and corners are the interior n cells away
    assert np.array_equal(out[0, 1:-1], out[n, 1:-1]) and np.array_equal(out[n + 1, 1:-1], out[1, 1:-1])
    assert np.array_equal(out[1:-1, 0], out[1:-1, n]) and np.array_equal(out[1:-1, n + 1], out[1:-1, 1])
    assert out[0, 0] == out[n, n] and out[0, n + 1] == out[n, 1]
    assert out[n + 1, 0] == out[1, n] and out[n + 1, n + 1] == out[1, 1]


def test_periodic_checkerboard_factor_is_one_minus_two_omega():
    """(p, q) = (n/2, n/2): the checkerboard, damped by 1 - 2 omega = -1/3 per sweep."""
    n, N = 12, 7
    h, lam = lam_of(n)
    i = np.arange(1, n + 1)[:, None]
    j = np.arange(1, n + 1)[None, :]
    board = (-1.0) ** (i + j)
    out, _, _ = oracle.relax(W.embed(board, n, n + 2), np.zeros((n, n)), n, h, lam, N,
                             bc=oracle.BC_PERIODIC, resmode=oracle.RES_NONE)
    np.testing.assert_allclose(out[1:-1, 1:-1], (1 - 2 * OMEGA) ** N * board, rtol=0, atol=1e-15)


def test_periodic_sweeps_match_dense_circulant_iteration():
    n, N = 7, 20
    h, lam = lam_of(n)
    f = W.uniform_rhs(n, 71)
    phi0 = W.uniform_phi(n, 72)
    out, mx, sq = oracle.relax(phi0, f, n, h, lam, N, bc=oracle.BC_PERIODIC)
    A = torus_laplacian(n, h)
    x = phi0[1:-1, 1:-1].ravel().copy()
    for _ in range(N):
        x = x + lam * (A @ x) - lam * f.ravel()
    assert np.abs(out[1:-1, 1:-1].ravel() - x).max() <= 1e-13 * np.abs(x).max()
    r = f.ravel() - A @ x
    assert mx == pytest.approx(np.abs(r).max(), rel=1e-10)
    assert sq == pytest.approx(np.sum(r * r), rel=1e-10)
    r_or, mx2, _ = oracle.residual(out, f, n, h, bc=oracle.BC_PERIODIC)
    assert np.abs(r_or.ravel() - r).max() <= 1e-10 * np.abs(r).max()


def test_periodic_constant_is_fixed_and_mean_moves_by_lambda_mean_f():
    """S of a constant is exactly 0 on a torus, so a constant is a fixed point for f = 0;
    and sum(S phi) = 0, so each sweep lowers the sum of phi by lambda * sum(f) (up to
    rounding)."""
    n = 20
    h, lam = lam_of(n)
    c = np.full((n + 2, n + 2), 0.625)
    out, _, _ = oracle.relax(c, np.zeros((n, n)), n, h, lam, 9, bc=oracle.BC_PERIODIC,
                             resmode=oracle.RES_NONE)
    assert np.all(out == 0.625)
    f = W.uniform_rhs(n, 73)
    phi0 = W.uniform_phi(n, 74)
    N = 15
    out, _, _ = oracle.relax(phi0, f, n, h, lam, N, bc=oracle.BC_PERIODIC, resmode=oracle.RES_NONE)
    expect = phi0[1:-1, 1:-1].sum() - N * lam * f.sum()
    assert out[1:-1, 1:-1].sum() == pytest.approx(expect, abs=1e-12 * n * n)


def test_periodic_stencil_of_mode_is_its_eigenvalue():
    n, p, q = 24, 5, 2
    h = 1.0 / n
    mode = periodic_mode(n, p, q)
    s = oracle.apply_stencil(W.embed(mode, n, n + 2), n, bc=oracle.BC_PERIODIC)
    ev = -4.0 * (np.sin(np.pi * p / n) ** 2 + np.sin(np.pi * q / n) ** 2)
    # the mode's samples carry the rounding of cos at arguments up to ~40: a few 1e-15
    # each, times the stencil's weights (sum 8)
    np.testing.assert_allclose(s, ev * mode, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_residual_terms_are_the_norms_terms(dt):
    """The per-cell residuals behind the exact sum of squares are the numbers the norm
    pass takes: their max magnitude is the oracle's max|r| bit for bit, they equal the
    stored residual in FP64 and FP32 (and round to it in BF16), and their squares summed
    exactly (math.fsum) lie within the recursive-summation bound of the oracle's own
    row-major sum; the exact sum keeps what a sequential sum loses past 2^53."""
    n = 45
    h, _ = lam_of(n)
    phi = W.uniform_phi(n, 25)
    f = W.uniform_rhs(n, 26)
    if dt == "f64":
        p, q = phi, f
    elif dt == "f32":
        p, q = phi.astype(np.float32), f.astype(np.float32)
    else:
        p, q = oracle.f32_to_bf16_bits(phi.astype(np.float32)), oracle.f32_to_bf16_bits(f.astype(np.float32))
    r, mx, sq = oracle.residual(p, q, n, h)
    rd, mx2, sq2 = oracle.residual_terms(p, q, n, h)
    assert (mx2, sq2) == (mx, sq)
    assert np.abs(rd).max() == mx
    if dt == "bf16":
        assert np.array_equal(oracle.f32_to_bf16_bits(rd.astype(np.float32)), r)
    else:
        assert np.array_equal(rd.view(np.int64), r.astype(np.float64).view(np.int64))
    ex = oracle.exact_sum_squares(rd)
    u = 2.0 ** -53
    assert abs(sq - ex) <= (n * n) * u * ex
    # squares 2^54 and four 1s: a sequential double sum stays at 2^54 (ulp 4), the exact
    # sum 2^54 + 4 is representable
    terms = np.array([2.0 ** 27, 1.0, 1.0, 1.0, 1.0])
    seq = 0.0
    for t in terms:
        seq += t * t
    assert seq == 2.0 ** 54 and oracle.exact_sum_squares(terms) == 2.0 ** 54 + 4.0


# ------------------------------------------------------------- box domains --

def _split(grid, nbx, nby, n):
    """A ghosted domain grid cut into ghosted boxes (each box's ghost ring from the domain)."""
    return [np.ascontiguousarray(grid[bi * n:bi * n + n + 2, bj * n:bj * n + n + 2])
            for bi in range(nby) for bj in range(nbx)]


@pytest.mark.parametrize("bc", [oracle.BC_DIRICHLET0, oracle.BC_GHOST_FIXED, oracle.BC_PERIODIC])
@pytest.mark.parametrize("nbx,nby", [(2, 2), (3, 1), (1, 2)])
def test_boxes_with_exchange_every_sweep_equal_the_whole_domain(bc, nbx, nby):
    """Section IV's boxes: exchanging the ghost layers before every sweep, then relaxing each
    box with its ghosts held, is the Jacobi sweep of the whole domain -- bit for bit, for
    each boundary rule (with fixed ghosts the domain's own ghost ring is what the boxes on
    its edge hold)."""
    n, N = 12, 9
    Ny, Nx = nby * n, nbx * n
    rng = np.random.default_rng(70 + 3 * nbx + nby)
    dom = np.zeros((Ny + 2, Nx + 2))
    dom[1:Ny + 1, 1:Nx + 1] = rng.uniform(-1, 1, (Ny, Nx))
    dom[0, :] = rng.uniform(-1, 1, Nx + 2)
    dom[Ny + 1, :] = rng.uniform(-1, 1, Nx + 2)
    dom[:, 0] = rng.uniform(-1, 1, Ny + 2)
    dom[:, Nx + 1] = rng.uniform(-1, 1, Ny + 2)
    F = rng.uniform(-1, 1, (Ny, Nx))
    if bc == oracle.BC_PERIODIC:
        F -= F.mean()
    h = 1.0 / Nx
    lam = (2.0 / 3.0) * h * h / 4.0
    # boxes on the domain's edge start with the domain's ghost ring there (what GHOST_FIXED
    # keeps; the other rules overwrite it)
    boxes = _split(dom, nbx, nby, n)
    fs = [np.ascontiguousarray(F[bi * n:(bi + 1) * n, bj * n:(bj + 1) * n]) for bi in range(nby) for bj in range(nbx)]
    got = oracle.relax_boxes(boxes, fs, nbx, nby, n, h, lam, N, exchange=1, bc=bc)
    ref = _rect_reference(dom, F, Ny, Nx, h, lam, N, bc)
    if Nx == Ny:
        # the written-out rectangle sweep is the oracle's sweep on square domains
        sq, _, _ = oracle.relax(dom, F, Ny, h, lam, N, bc=bc, resmode=oracle.RES_NONE)
        assert np.array_equal(sq[1:Ny + 1, 1:Nx + 1], ref[1:Ny + 1, 1:Nx + 1])
    for b, g in enumerate(got):
        bi, bj = divmod(b, nbx)
        want = ref[bi * n + 1:bi * n + n + 1, bj * n + 1:bj * n + n + 1]
        assert np.array_equal(g[1:n + 1, 1:n + 1].view(np.int64), want.view(np.int64)), (b, bc)


def _rect_reference(dom, F, Ny, Nx, h, lam, N, bc):
    """N Jacobi sweeps of a rectangular domain: the three steps written out (ghosts per bc,
    stencil in the paper's order, update into a separate array)."""
    c = 1.0 / (h * h)
    w = lam / (h * h)
    phi = dom.copy()
    for _ in range(N):
        g = phi.copy()
        if bc == oracle.BC_DIRICHLET0:
            g[0, 1:Nx + 1] = -g[1, 1:Nx + 1]
            g[Ny + 1, 1:Nx + 1] = -g[Ny, 1:Nx + 1]
            g[1:Ny + 1, 0] = -g[1:Ny + 1, 1]
            g[1:Ny + 1, Nx + 1] = -g[1:Ny + 1, Nx]
        elif bc == oracle.BC_PERIODIC:
            g[0, 1:Nx + 1] = g[Ny, 1:Nx + 1]
            g[Ny + 1, 1:Nx + 1] = g[1, 1:Nx + 1]
            g[1:Ny + 1, 0] = g[1:Ny + 1, Nx]
            g[1:Ny + 1, Nx + 1] = g[1:Ny + 1, 1]
        C = g[1:Ny + 1, 1:Nx + 1]
        s = (((g[0:Ny, 1:Nx + 1] - 4.0 * C) + g[1:Ny + 1, 0:Nx]) + g[1:Ny + 1, 2:Nx + 2]) + g[2:Ny + 2, 1:Nx + 1]
        new = phi.copy()
        new[1:Ny + 1, 1:Nx + 1] = (C + w * s) - lam * F
        phi = new
    return phi


def test_boxes_with_lagged_exchange_hold_interfaces_between_exchanges():
    """Exchanging every k > 1 sweeps differs from the whole-domain sweep only through the
    held interface values: the first sweep after an exchange is exact, and one box with
    its ghost ring refreshed is exactly the fixed-ghost relaxation of that box."""
    n = 10
    rng = np.random.default_rng(80)
    boxes = [np.zeros((n + 2, n + 2)) for _ in range(2)]
    for b in boxes:
        b[1:n + 1, 1:n + 1] = rng.uniform(-1, 1, (n, n))
    fs = [rng.uniform(-1, 1, (n, n)) for _ in range(2)]
    h = 1.0 / (2 * n)
    lam = (2.0 / 3.0) * h * h / 4.0
    one = oracle.relax_boxes(boxes, fs, 2, 1, n, h, lam, 1, exchange=1)
    lagged = oracle.relax_boxes(boxes, fs, 2, 1, n, h, lam, 4, exchange=4)
    exact4 = oracle.relax_boxes(boxes, fs, 2, 1, n, h, lam, 4, exchange=1)
    # k = 4: every ghost (interface and domain edge) is held for sweeps 2..4, so a held value
    # reaches 3 cells in; cells farther from every ghost see none of them
    far = slice(4, n - 3 + 1)
    for l4, e4 in zip(lagged, exact4):
        assert np.array_equal(l4[far, far], e4[far, far])
    assert not np.array_equal(lagged[0][1:n + 1, n], exact4[0][1:n + 1, n])  # next to the interface
    # one sweep with a fresh exchange is the whole-domain sweep (same as exchange = 1)
    first = oracle.relax_boxes(boxes, fs, 2, 1, n, h, lam, 1, exchange=1)
    assert all(np.array_equal(a, b) for a, b in zip(one, first))
