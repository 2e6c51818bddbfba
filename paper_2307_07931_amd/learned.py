"""Training of the learned correction network on the GPU.

Argument marshalling over the C ABI only: training pairs come from plain fused
relaxation (``px_relax_fused``) and ``px_net_make_pair``; forward, loss, backward and
Adam run in the library's kernels (``px_net_loss_grad``, ``px_net_adam``).  PyTorch
holds the device buffers and assembles mini-batches by indexing.

Pairs.  The error of damped Jacobi evolves by e <- (I - lambda L) e whatever the
right-hand side is, so the (residual, error) pairs of plain solves are those of the
homogeneous problem L phi = 0 started from phi0 = -e0 (exact solution 0, error -phi,
residual -L phi).  The caller draws the initial errors (e.g. with the |k|^-3
amplitude spectrum of L^-1 f for a right-hand side f with |k|^-2 power) and passes
them in; snapshots are taken after the given numbers of sweeps.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import (BC_DIRICHLET0, LOSS_MSE, RES_NONE, Context, Net, alloc_grid, alloc_rhs, make_pair,
               relax_fused)

OMEGA = 2.0 / 3.0
SNAPSHOTS = (16, 64, 256, 1024, 4096, 16384)


def training_pairs(fields, ctx: Context, snapshots=SNAPSHOTS, loss=LOSS_MSE, tblock=0):
    """fields: sequence of n x n float64 arrays (initial errors).  Returns device float32
    tensors X, T of shape (len(fields) * len(snapshots), n, n): normalised residuals and
    normalised errors after each snapshot's number of plain sweeps."""
    n = fields[0].shape[0]
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    P = len(fields) * len(snapshots)
    X = torch.empty((P, n, n), dtype=torch.float32, device="cuda")
    T = torch.empty_like(X)
    f = alloc_rhs(n)
    a, b = alloc_grid(n), alloc_grid(n)
    k = 0
    for fld in fields:
        a.zero_()
        a[1:n + 1, 1:n + 1] = torch.from_numpy(np.ascontiguousarray(fld, dtype=np.float64)).to("cuda")
        done = 0
        for m in snapshots:
            if m > done:
                relax_fused(a, b, n, f, h, lam, m - done, ctx, tblock=tblock, bc=BC_DIRICHLET0,
                            resmode=RES_NONE)
                a, b = b, a
                done = m
            make_pair(a, n, X[k], T[k], ctx, loss=loss)
            k += 1
    return X, T


def train(net: Net, X, T, steps: int, batch: int = 2, lr: float = 1e-3, loss=LOSS_MSE, seed: int = 0,
          log_every: int = 50, lr_final: float | None = None):
    """Adam on mini-batches of whole images drawn (seeded) from the pairs X, T.  The
    learning rate decays by a cosine from lr to lr_final (default lr / 20).  Returns the
    losses read every log_every steps (and at the last step)."""
    g = torch.Generator().manual_seed(seed)
    lr_final = lr / 20.0 if lr_final is None else lr_final
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    log = []
    for it in range(steps):
        idx = torch.randperm(X.shape[0], generator=g)[:batch].to("cuda")
        x = X.index_select(0, idx).contiguous()
        t = T.index_select(0, idx).contiguous()
        want = (it % log_every == 0) or it == steps - 1
        net.loss_grad(x, t, loss=loss, loss_out=out if want else None)
        rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * it / max(1, steps - 1)))
        net.adam(rate)
        if want:
            log.append((it, float(out.item())))
    return log
