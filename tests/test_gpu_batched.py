"""Batched relaxation and batched mixed-precision solves on the GPU: every member of a
batch must equal its single-problem run bit for bit (and so the oracle)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_07931_amd as px
import workloads as W

import helpers as H

pytestmark = pytest.mark.gpu
OMEGA = 2.0 / 3.0


@pytest.fixture(scope="module")
def ctx():
    H.require_gpu()
    c = px.Context()
    yield c
    c.close()


SIZES = [1, 2, 7, 33, 64, 127, 130, 257, 64, 5, 300, 96]


@pytest.mark.parametrize("dt,tblock,nsweeps", [("f64", 4, 13), ("f32", 8, 21), ("bf16", 3, 10), ("f64", 1, 3),
                                               ("f64", 8, 24)])
def test_relax_batched_equals_single_and_oracle(ctx, dt, tblock, nsweeps):
    items, refs = [], []
    for k, n in enumerate(SIZES):
        h = 1.0 / n
        lam = OMEGA * h * h / 4.0
        phi0 = W.uniform_phi(n, 700 + k)
        f = W.uniform_rhs(n, 800 + k)
        items.append((H.device_grid(phi0, n, dt), H.device_rhs(f, n, dt), n, h, lam))
        refs.append((phi0, f, n, h, lam))
    norms = torch.full((2 * len(items),), float("nan"), dtype=torch.float64, device="cuda")
    print(f"case: batch {dt} tblock={tblock} sweeps={nsweeps} sizes={SIZES}", flush=True)
    px.relax_batched(items, nsweeps, ctx, tblock=tblock, norms=norms)
    torch.cuda.synchronize()
    nm = norms.cpu().numpy()
    for k, ((phi, _, n, _, _), (phi0, f, _, h, lam)) in enumerate(zip(items, refs)):
        ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, nsweeps, dt)
        H.assert_grid_bitwise(H.to_storage_np(phi, dt), ref, n, what=f"member {k} (n={n})")
        H.assert_norms(nm[2 * k:2 * k + 2], mx, sq, n=n)


@pytest.mark.parametrize("mode,inner", [(px.SOLVE_MIXED_F32, 32), (px.SOLVE_MIXED_BF16, 16)])
def test_solve_batched_equals_single_solves(ctx, mode, inner):
    sizes = [16, 24, 33, 40, 17, 64, 48, 20]
    items, singles = [], []
    for k, n in enumerate(sizes):
        h = 1.0 / n
        lam = OMEGA * h * h / 4.0
        f = W.grf_rhs(n, 900 + k)
        if k == 3:
            f[:] = 0.0  # converged before the first step (residual 0 <= tol * 0)
        items.append((H.device_grid(np.zeros((n + 2, n + 2)), n, "f64"), H.device_rhs(f, n, "f64"), n, h, lam))
        phi = H.device_grid(np.zeros((n + 2, n + 2)), n, "f64")
        st = px.solve(phi, n, H.device_rhs(f, n, "f64"), h, lam, ctx, mode=mode, rtol=1e-9,
                      inner_sweeps=inner, tblock=8)
        singles.append((phi, st))
    status, stats = px.solve_batched(items, ctx, mode=mode, rtol=1e-9, inner_sweeps=inner, tblock=8)
    assert status == px.OK
    for k, ((phi, _, n, _, _), (sphi, sst), bst) in enumerate(zip(items, singles, stats)):
        assert bst.outer_steps == sst.outer_steps and bst.sweeps == sst.sweeps, (k, bst, sst)
        assert bst.res_max == sst.res_max
        inner_mask = np.zeros((n + 2, n + 2), dtype=bool)
        inner_mask[1:n + 1, 1:n + 1] = True
        H.assert_grid_bitwise(H.to_storage_np(phi, "f64"), H.to_storage_np(sphi, "f64"), n, mask=inner_mask,
                              what=f"member {k} (n={n})")
    # replaying the same captured step again from zero gives the same result
    for phi, _, n, _, _ in items:
        phi.zero_()
    status2, stats2 = px.solve_batched(items, ctx, mode=mode, rtol=1e-9, inner_sweeps=inner, tblock=8)
    assert status2 == px.OK and [s.sweeps for s in stats2] == [s.sweeps for s in stats]


def test_solve_batched_reports_budget(ctx):
    n = 32
    h = 1.0 / n
    items = [(H.device_grid(np.zeros((n + 2, n + 2)), n, "f64"), H.device_rhs(W.grf_rhs(n, 77), n, "f64"), n, h,
              OMEGA * h * h / 4.0)]
    status, stats = px.solve_batched(items, ctx, rtol=1e-12, max_sweeps=64, inner_sweeps=32, raise_on_error=False)
    assert status == px.ENOTCONV and stats[0].sweeps == 64


def test_autotuned_batch_gives_identical_results():
    """After px_autotune_batched (tile rows per size, sweeps per launch) a batched relax and
    a batched solve with tblock 0 use the tuned configuration and give the oracle's / the
    single solves' results bit for bit."""
    H.require_gpu()
    c = px.Context()
    sizes = [40, 100, 40, 257, 100, 64]
    scratch = []
    for k, n in enumerate(sizes):
        h = 1.0 / n
        scratch.append((H.device_grid(W.uniform_phi(n, 950 + k), n, "f32"),
                        H.device_rhs(W.uniform_rhs(n, 960 + k), n, "f32"), n, h, OMEGA * h * h / 4.0))
    kbest = px.autotune_batched(scratch, c)
    print(f"tuned batch: k={kbest}", flush=True)
    assert 1 <= kbest <= 8
    items, refs = [], []
    for k, n in enumerate(sizes):
        h = 1.0 / n
        lam = OMEGA * h * h / 4.0
        phi0 = W.uniform_phi(n, 970 + k)
        f = W.uniform_rhs(n, 980 + k)
        items.append((H.device_grid(phi0, n, "f32"), H.device_rhs(f, n, "f32"), n, h, lam))
        refs.append((phi0, f, n, h, lam))
    norms = torch.zeros(2 * len(items), dtype=torch.float64, device="cuda")
    px.relax_batched(items, 19, c, tblock=0, norms=norms)
    torch.cuda.synchronize()
    nm = norms.cpu().numpy()
    for k, ((phi, _, n, _, _), (phi0, f, _, h, lam)) in enumerate(zip(items, refs)):
        ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, 19, "f32")
        H.assert_grid_bitwise(H.to_storage_np(phi, "f32"), ref, n, what=f"member {k} (n={n})")
        H.assert_norms(nm[2 * k:2 * k + 2], mx, sq, n=n)
    sol, singles = [], []
    for k, n in enumerate(sizes):
        h = 1.0 / n
        lam = OMEGA * h * h / 4.0
        f = W.grf_rhs(n, 990 + k)
        sol.append((H.device_grid(np.zeros((n + 2, n + 2)), n, "f64"), H.device_rhs(f, n, "f64"), n, h, lam))
        phi = H.device_grid(np.zeros((n + 2, n + 2)), n, "f64")
        singles.append((phi, px.solve(phi, n, H.device_rhs(f, n, "f64"), h, lam, c, mode=px.SOLVE_MIXED_F32,
                                      rtol=1e-7, inner_sweeps=32, tblock=8)))
    status, stats = px.solve_batched(sol, c, mode=px.SOLVE_MIXED_F32, rtol=1e-7, inner_sweeps=32, tblock=0)
    assert status == px.OK
    for k, ((phi, _, n, _, _), (sphi, sst), bst) in enumerate(zip(sol, singles, stats)):
        assert bst.sweeps == sst.sweeps, (k, bst, sst)
        m = np.zeros((n + 2, n + 2), dtype=bool)
        m[1:n + 1, 1:n + 1] = True
        H.assert_grid_bitwise(H.to_storage_np(phi, "f64"), H.to_storage_np(sphi, "f64"), n, mask=m,
                              what=f"solve member {k} (n={n})")
    c.close()
