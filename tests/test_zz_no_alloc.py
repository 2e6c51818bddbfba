"""px_relax_fused_noalloc (one launch, reduction partials in the library's fixed
device array) against px_relax_fused with a context, through the C ABI: the same
output grid and norms bit for bit, on calls in a row that reuse the fixed array --
a large grid first, then smaller ones (stale partials of the earlier call beyond the
later call's count must not be read), across precisions, boundary rules and
residual modes.  The first case is also compared with the oracle."""
import numpy as np
import pytest
import torch

import paper_2307_07931_amd as px
import workloads as W

import helpers as H

pytestmark = pytest.mark.gpu
OMEGA = 2.0 / 3.0

# (n, dtype, sweeps, resmode, bc), run in this order
CALLS = [(777, "f64", 8, px.RES_FINAL, px.BC_DIRICHLET0),
         (130, "f32", 5, px.RES_LAGGED, px.BC_PERIODIC),
         (64, "bf16", 3, px.RES_FINAL, px.BC_GHOST_FIXED),
         (300, "f64", 1, px.RES_NONE, px.BC_DIRICHLET0)]


def test_noalloc_equals_context_entry_point_on_calls_in_a_row():
    H.require_gpu()
    ctx = px.Context()
    for i, (n, dt, k, rm, bc) in enumerate(CALLS):
        h = 1.0 / n
        lam = OMEGA * h * h / 4.0
        phi0 = W.uniform_phi(n, 7100 + i)
        f = W.uniform_rhs(n, 7200 + i)
        pin = H.device_grid(phi0, n, dt)
        fd = H.device_rhs(f, n, dt)
        out_ctx = torch.full_like(pin, H.SENTINEL)
        out_na = torch.full_like(pin, H.SENTINEL)
        nm_ctx = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        nm_na = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        print(f"case {i}: noalloc n={n} {dt} sweeps={k} res={rm} bc={bc}", flush=True)
        px.relax_fused(pin, out_ctx, n, fd, h, lam, k, ctx, tblock=k, bc=bc, resmode=rm, norms=nm_ctx)
        px.relax_fused_noalloc(pin, out_na, n, fd, h, lam, k, bc=bc, resmode=rm,
                               norms=nm_na if rm != px.RES_NONE else None)
        torch.cuda.synchronize()
        a, b = H.to_storage_np(out_ctx, dt), H.to_storage_np(out_na, dt)
        assert np.array_equal(H.bits(a), H.bits(b)), f"case {i}: grids differ"
        if rm != px.RES_NONE:
            x, y = nm_ctx.cpu().numpy(), nm_na.cpu().numpy()
            assert np.array_equal(x.view(np.int64), y.view(np.int64)), (i, x, y)
        else:
            assert torch.isnan(nm_na).all()
        if i == 0:
            ref, mx, sq = H.oracle_relax(phi0, f, n, h, lam, k, dt, bc=bc, resmode=rm)
            H.assert_grid_bitwise(b, ref, n, what="noalloc vs oracle")
            H.assert_norms(nm_na.cpu().numpy(), mx, sq, n=n)
    ctx.close()


def test_noalloc_rejects_oversized_grid_and_sweep_counts():
    H.require_gpu()
    n = 64
    pin = px.alloc_grid(n)
    pout = torch.zeros_like(pin)
    fd = px.alloc_rhs(n)
    norms = torch.zeros(2, dtype=torch.float64, device="cuda")
    for k in (0, 9):
        with pytest.raises(px.ProtoxError):
            px.relax_fused_noalloc(pin, pout, n, fd, 1 / n, 1e-5, k, norms=norms)
