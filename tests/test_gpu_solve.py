"""px_solve on the GPU: plain relaxation to a tolerance, mixed-precision refinement
(FP32 / BF16 inner sweeps, FP64 outer residual and update) against the oracle's
refinement, and the failure statuses."""
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


def setup(n, f, dt="f64"):
    phi = H.device_grid(np.zeros((n + 2, n + 2)), n, dt)
    fd = H.device_rhs(f, n, dt)
    h = 1.0 / n
    return phi, fd, h, OMEGA * h * h / 4.0


def test_plain_solve_equals_oracle_sweeps(ctx):
    """Plain solve checks every `check_every` sweeps; its iterate is the oracle's after the
    same number of sweeps, bit for bit, and the stopping rule holds."""
    n = 48
    f = W.grf_rhs(n, 101)
    phi, fd, h, lam = setup(n, f)
    st = px.solve(phi, n, fd, h, lam, ctx, mode=px.SOLVE_PLAIN, rtol=1e-6, check_every=50, tblock=8)
    assert st.status == px.OK and st.sweeps % 50 == 0 and st.rel_res_max <= 1e-6
    ref, mx, _ = oracle.relax(np.zeros((n + 2, n + 2)), f, n, h, lam, st.sweeps)
    H.assert_grid_bitwise(H.to_storage_np(phi, "f64"), ref, n)
    assert st.res_max == mx
    _, mx_prev, _ = oracle.relax(np.zeros((n + 2, n + 2)), f, n, h, lam, st.sweeps - 50)
    assert mx_prev > 1e-6 * np.abs(f).max()  # it did not stop late


@pytest.mark.parametrize("mode,lowp,k_in", [(px.SOLVE_MIXED_F32, 1, 64), (px.SOLVE_MIXED_BF16, 2, 16)])
def test_mixed_solve_equals_oracle_refinement(ctx, mode, lowp, k_in):
    n = 40
    f = W.grf_rhs(n, 102)
    phi, fd, h, lam = setup(n, f)
    st = px.solve(phi, n, fd, h, lam, ctx, mode=mode, rtol=1e-11, inner_sweeps=k_in, tblock=8)
    assert st.status == px.OK and st.rel_res_max <= 1e-11
    ref = np.zeros((n + 2, n + 2))
    steps, mx, _ = oracle.refine(ref, f, n, h, lam, lowp, k_in, 100000, 1e-11)
    assert st.outer_steps == steps
    inner = np.zeros((n + 2, n + 2), dtype=bool)
    inner[1:n + 1, 1:n + 1] = True
    H.assert_grid_bitwise(H.to_storage_np(phi, "f64"), ref, n, mask=inner)
    assert st.res_max == mx
    ex = exact.dst_solve(f, h)
    assert np.abs(H.to_storage_np(phi, "f64")[1:n + 1, 1:n + 1] - ex).max() <= 1e-10 * np.abs(ex).max()


def test_mixed_solve_matches_plain_rate(ctx):
    """With the inner solves restarted every k_in sweeps the refined iteration needs no
    more sweeps than plain FP64 relaxation (up to one inner block)."""
    n = 32
    f = W.uniform_rhs(n, 103)
    phi, fd, h, lam = setup(n, f)
    p = px.solve(phi, n, fd, h, lam, ctx, mode=px.SOLVE_PLAIN, rtol=1e-9, check_every=16)
    phi2, fd2, _, _ = setup(n, f)
    m = px.solve(phi2, n, fd2, h, lam, ctx, mode=px.SOLVE_MIXED_F32, rtol=1e-9, inner_sweeps=16)
    assert m.sweeps <= p.sweeps + 16


def test_nonfinite_rhs_is_reported(ctx):
    n = 20
    f = W.uniform_rhs(n, 104)
    f[3, 3] = np.inf
    phi, fd, h, lam = setup(n, f)
    st = px.solve(phi, n, fd, h, lam, ctx, rtol=1e-8, raise_on_error=False)
    assert st.status == px.ENONFINITE


def test_divergence_is_reported(ctx):
    """omega = 1.5 > 1 makes the highest modes grow (factor 1 - 2 omega = -2)."""
    n = 24
    f = W.uniform_rhs(n, 105)
    phi, fd, h, _ = setup(n, f)
    lam = 1.5 * h * h / 4.0
    st = px.solve(phi, n, fd, h, lam, ctx, rtol=1e-12, check_every=10, raise_on_error=False)
    assert st.status == px.EDIVERGED


def test_sweep_budget_is_reported(ctx):
    n = 64
    f = W.uniform_rhs(n, 106)
    phi, fd, h, lam = setup(n, f)
    st = px.solve(phi, n, fd, h, lam, ctx, rtol=1e-12, max_sweeps=200, check_every=100,
                  raise_on_error=False)
    assert st.status == px.ENOTCONV and st.sweeps == 200
    with pytest.raises(px.ProtoxError):
        px.solve(phi, n, fd, h, lam, ctx, rtol=1e-12, max_sweeps=100, check_every=100)


@pytest.mark.parametrize("mode", [px.SOLVE_MIXED_F32, px.SOLVE_MIXED_BF16])
def test_mixed_graph_path_equals_host_loop(ctx, mode):
    """Mixed solves of grids up to 1024^2 with 16-byte aligned rows run as a graph-replayed
    batch of one; a layout that does not qualify runs the host-driven loop.  Same sweeps,
    outer steps, norms and iterate, bit for bit."""
    n = 48
    f = W.grf_rhs(n, 107)
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    phi_a = H.device_grid(np.zeros((n + 2, n + 2)), n, "f64")              # 16-byte rows: graph
    phi_b = H.device_grid(np.zeros((n + 2, n + 2)), n, "f64", ld=n + 3)    # odd pitch: host loop
    fd = H.device_rhs(f, n, "f64")
    a = px.solve(phi_a, n, fd, h, lam, ctx, mode=mode, rtol=1e-9, inner_sweeps=24, tblock=8)
    b = px.solve(phi_b, n, fd, h, lam, ctx, mode=mode, rtol=1e-9, inner_sweeps=24, tblock=8)
    assert (a.sweeps, a.outer_steps, a.res_max) == (b.sweeps, b.outer_steps, b.res_max)
    m = np.zeros((n + 2, n + 2), dtype=bool)
    m[1:n + 1, 1:n + 1] = True
    H.assert_grid_bitwise(H.to_storage_np(phi_a, "f64"), H.to_storage_np(phi_b, "f64"), n, mask=m)


def test_mixed_failure_statuses(ctx):
    n = 24
    h = 1.0 / n
    f = W.uniform_rhs(n, 108)
    bad = f.copy()
    bad[5, 7] = np.nan
    for layout in (None, n + 3):  # graph path, host loop
        phi = H.device_grid(np.zeros((n + 2, n + 2)), n, "f64", ld=layout)
        st = px.solve(phi, n, H.device_rhs(bad, n, "f64"), h, OMEGA * h * h / 4, ctx, mode=px.SOLVE_MIXED_F32,
                      rtol=1e-8, raise_on_error=False)
        assert st.status == px.ENONFINITE, layout
        phi = H.device_grid(np.zeros((n + 2, n + 2)), n, "f64", ld=layout)
        st = px.solve(phi, n, H.device_rhs(f, n, "f64"), h, OMEGA * h * h / 4, ctx, mode=px.SOLVE_MIXED_F32,
                      rtol=1e-14, max_sweeps=96, inner_sweeps=32, raise_on_error=False)
        assert st.status == px.ENOTCONV and st.sweeps == 96, layout
        phi = H.device_grid(np.zeros((n + 2, n + 2)), n, "f64", ld=layout)
        st = px.solve(phi, n, H.device_rhs(f, n, "f64"), h, 1.5 * h * h / 4, ctx, mode=px.SOLVE_MIXED_F32,
                      rtol=1e-14, inner_sweeps=32, raise_on_error=False)
        assert st.status in (px.EDIVERGED, px.ENONFINITE), (layout, st)


@pytest.mark.parametrize("mode,inner,slack", [(px.SOLVE_MIXED_F32, 1024, 1.01), (px.SOLVE_MIXED_BF16, 128, 1.05)])
def test_default_inner_converges_like_plain_fp64(ctx, mode, inner, slack):
    """The default inner solves (1024 FP32 or 128 BF16 sweeps per FP64 step) reach
    max|r| <= 1e-10 max|f| in about the sweeps plain FP64 relaxation needs -- the property
    the time-to-tolerance comparison at large grids rests on -- with the error against the
    exact discrete solution of the same size, and equal an explicit inner count of the same
    size bit for bit."""
    n = 128
    f = W.grf_rhs(n, 109)
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    fd = H.device_rhs(f, n, "f64")
    grids = [H.device_grid(np.zeros((n + 2, n + 2)), n, "f64") for _ in range(3)]
    print(f"case: n={n} mode={mode} default inner vs plain FP64 and inner={inner}", flush=True)
    plain = px.solve(grids[0], n, fd, h, lam, ctx, mode=px.SOLVE_PLAIN, rtol=1e-10)
    mixed = px.solve(grids[1], n, fd, h, lam, ctx, mode=mode, rtol=1e-10)
    explicit = px.solve(grids[2], n, fd, h, lam, ctx, mode=mode, rtol=1e-10, inner_sweeps=inner)
    assert mixed.rel_res_max <= 1e-10
    assert mixed.sweeps <= slack * plain.sweeps + inner, (mixed.sweeps, plain.sweeps)
    assert mixed.sweeps % inner == 0
    assert (mixed.sweeps, mixed.res_max) == (explicit.sweeps, explicit.res_max)
    assert torch.equal(grids[1], grids[2])
    ex = exact.dst_solve(f, h)
    for g in grids[:2]:
        err = np.abs(H.to_storage_np(g, "f64")[1:n + 1, 1:n + 1] - ex).max() / np.abs(ex).max()
        assert err < 1e-8
