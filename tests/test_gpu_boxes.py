"""A domain split into boxes (Section IV: boxes with their own ghost layers, the ghost
cells copied from the neighbouring boxes' interiors between sweeps) on the GPU:
px_relax_boxes against px_relax_fused on the whole domain (exchange before every sweep)
and against the oracle's box relaxation (exchange every k sweeps), bit for bit on every
box interior."""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_07931_amd as px
import workloads as W

import helpers as H

pytestmark = pytest.mark.gpu
OMEGA = 2.0 / 3.0


def domain(nbx, nby, n, seed, periodic):
    Ny, Nx = nby * n, nbx * n
    rng = np.random.default_rng(seed)
    dom = rng.uniform(-1, 1, (Ny + 2, Nx + 2))  # interior and a ghost ring (held by GHOST_FIXED)
    F = rng.uniform(-1, 1, (Ny, Nx))
    if periodic:
        F -= F.mean()
    return dom, F


def split(dom, F, nbx, nby, n):
    boxes = [np.ascontiguousarray(dom[bi * n:bi * n + n + 2, bj * n:bj * n + n + 2])
             for bi in range(nby) for bj in range(nbx)]
    fs = [np.ascontiguousarray(F[bi * n:(bi + 1) * n, bj * n:(bj + 1) * n]) for bi in range(nby) for bj in range(nbx)]
    return boxes, fs


def gpu_boxes(boxes, fs, nbx, nby, n, h, lam, nsweeps, exchange, bc, dt, ctx):
    items = [(H.device_grid(b, n, dt), H.device_rhs(f, n, dt), n, h, lam) for b, f in zip(boxes, fs)]
    px.relax_boxes(items, nbx, nby, nsweeps, ctx, exchange=exchange, bc=bc)
    torch.cuda.synchronize()
    return [H.to_storage_np(it[0], dt) for it in items]


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("bc", [px.BC_DIRICHLET0, px.BC_GHOST_FIXED, px.BC_PERIODIC])
@pytest.mark.parametrize("nb,n", [(2, 64), (4, 64), (3, 33)])
def test_exchange_every_sweep_equals_whole_domain(dt, bc, nb, n):
    """Exchanging before every sweep makes the boxes one Jacobi sweep of the whole domain:
    equal to px_relax_fused on the assembled grid (4 x 4 boxes of 64^2 is the paper's
    256^2 domain of 64^2 boxes)."""
    H.require_gpu()
    N = nb * n
    h = 1.0 / N
    lam = OMEGA * h * h / 4.0
    dom, F = domain(nb, nb, n, 8000 + nb * 10 + n + bc, bc == px.BC_PERIODIC)
    boxes, fs = split(dom, F, nb, nb, n)
    c = px.Context()
    print(f"case: boxes {nb}x{nb} of {n}^2 {dt} bc={bc} exchange=1 sweeps=7", flush=True)
    got = gpu_boxes(boxes, fs, nb, nb, n, h, lam, 7, 1, bc, dt, c)
    whole, _ = H.gpu_relax(dom, F, N, h, lam, 7, dt, c, tblock=3, bc=bc, resmode=px.RES_NONE)
    c.close()
    for b, g in enumerate(got):
        bi, bj = divmod(b, nb)
        want = whole[bi * n + 1:bi * n + n + 1, bj * n + 1:bj * n + n + 1]
        assert np.array_equal(H.bits(g[1:n + 1, 1:n + 1]), H.bits(want)), (b, dt, bc)


@pytest.mark.parametrize("k", [2, 5, 8])
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_lagged_exchange_matches_oracle(k, dt):
    """Exchange every k sweeps on rectangular layouts (2 x 3 and 3 x 2 boxes): every box
    equals the oracle's box relaxation bit for bit (interiors and the ghost rings the last
    exchange left)."""
    H.require_gpu()
    n = 40
    for li, (nbx, nby) in enumerate(((2, 3), (3, 2))):
        bc = (px.BC_DIRICHLET0, px.BC_PERIODIC)[li]
        Nx = nbx * n
        h = 1.0 / Nx
        lam = OMEGA * h * h / 4.0
        dom, F = domain(nbx, nby, n, 8100 + 7 * k + li, bc == px.BC_PERIODIC)
        boxes, fs = split(dom, F, nbx, nby, n)
        c = px.Context()
        print(f"case: boxes {nbx}x{nby} of {n}^2 {dt} bc={bc} exchange={k} sweeps={3 * k}", flush=True)
        got = gpu_boxes(boxes, fs, nbx, nby, n, h, lam, 3 * k, k, bc, dt, c)
        c.close()
        ob = [H.oracle_input(b, dt) for b in boxes]
        of = [H.oracle_input(f, dt) for f in fs]
        ref = oracle.relax_boxes(ob, of, nbx, nby, n, h, lam, 3 * k, exchange=k, bc=bc)
        for b, (g, r) in enumerate(zip(got, ref)):
            H.assert_grid_bitwise(g, r, n, what=f"box {b} ({nbx}x{nby}, k={k}, {dt})")
