"""CPU oracle of the learned correction network -- TEST INFRASTRUCTURE ONLY.

Not part of the paper: a small convolutional network that maps a (normalised)
residual to a correction, used inside a refinement loop.  Architecture:

    x (1 channel) -> conv3x3 1->32 -> ReLU -> conv3x3 32->32 -> ReLU
                  -> conv3x3 32->32 -> ReLU -> conv3x3 32->1 -> y

3x3 kernels, no bias, zero padding (outside the image every activation is 0).
Weights in C order: W1 (32,1,3,3), W2 (32,32,3,3), W3 (32,32,3,3), W4 (1,32,3,3)
= 19008 numbers.  Activations are (batch, H, W, C) arrays (channels last).

Precision model of the GPU kernels (BF16 in, FP32 accumulate): weights, the input
and every hidden activation are rounded to bfloat16 before they are used; sums are
taken here in FP64.  `bf16=False` switches all rounding off (pure FP64 network, used
for finite-difference pins).  Losses: mean squared error, or the mean energy
(y - t) K (y - t) with K the negated 5-point stencil under odd reflection.
"""
from __future__ import annotations

import numpy as np

SHAPES = ((32, 1, 3, 3), (32, 32, 3, 3), (32, 32, 3, 3), (1, 32, 3, 3))
SIZES = tuple(int(np.prod(s)) for s in SHAPES)
NPARAM = sum(SIZES)  # 19008


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def unflatten(w: np.ndarray):
    w = np.asarray(w, dtype=np.float64).ravel()
    assert w.size == NPARAM
    out, o = [], 0
    for s, n in zip(SHAPES, SIZES):
        out.append(w[o:o + n].reshape(s))
        o += n
    return out


def flatten(ws) -> np.ndarray:
    return np.concatenate([np.asarray(w, dtype=np.float64).ravel() for w in ws])


def conv3x3(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """y[b,i,j,co] = sum_{ci,a,c} w[co,ci,a,c] x[b, i+a-1, j+c-1, ci], zero outside."""
    B, H, W, _ = x.shape
    xp = np.zeros((B, H + 2, W + 2, x.shape[3]))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    y = np.zeros((B, H, W, w.shape[0]))
    for a in range(3):
        for c in range(3):
            y += xp[:, a:a + H, c:c + W, :] @ w[:, :, a, c].T
    return y


def conv3x3_input_grad(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient of conv3x3 with respect to its input (the transposed convolution)."""
    B, H, W, _ = dy.shape
    dyp = np.zeros((B, H + 2, W + 2, dy.shape[3]))
    dyp[:, 1:H + 1, 1:W + 1, :] = dy
    dx = np.zeros((B, H, W, w.shape[1]))
    for a in range(3):
        for c in range(3):
            # x[i+a-1] fed y[i]  =>  y[i'] with i' = i - a + 1 feeds dx[i]
            dx += dyp[:, 2 - a:2 - a + H, 2 - c:2 - c + W, :] @ w[:, :, a, c]
    return dx


def conv3x3_weight_grad(x: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """dW[co,ci,a,c] = sum over batch and pixels of dy[.,i,j,co] x[., i+a-1, j+c-1, ci]."""
    B, H, W, Ci = x.shape
    xp = np.zeros((B, H + 2, W + 2, Ci))
    xp[:, 1:H + 1, 1:W + 1, :] = x
    Co = dy.shape[3]
    dw = np.zeros((Co, Ci, 3, 3))
    d2 = dy.reshape(-1, Co)
    for a in range(3):
        for c in range(3):
            dw[:, :, a, c] = d2.T @ xp[:, a:a + H, c:c + W, :].reshape(-1, Ci)
    return dw


def forward(w_flat: np.ndarray, x: np.ndarray, bf16: bool = True):
    """x: (B, H, W) input.  Returns (y (B, H, W), cache of activations)."""
    rnd = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    W1, W2, W3, W4 = [rnd(w) for w in unflatten(w_flat)]
    a0 = rnd(x)[..., None]
    a1 = rnd(np.maximum(conv3x3(a0, W1), 0.0))
    a2 = rnd(np.maximum(conv3x3(a1, W2), 0.0))
    a3 = rnd(np.maximum(conv3x3(a2, W3), 0.0))
    y = conv3x3(a3, W4)[..., 0]
    return y, dict(a0=a0, a1=a1, a2=a2, a3=a3, W=(W1, W2, W3, W4), bf16=bf16)


def energy_operator(d: np.ndarray) -> np.ndarray:
    """K d per image of d (B, H, W): 4 d(i,j) minus its four neighbours, where a neighbour
    outside the image is taken as -d(i,j) (odd reflection across the edge, the
    homogeneous Dirichlet ghost).  K is the negated 5-point stencil: symmetric positive
    definite, so d K d is the (unscaled) energy norm of d."""
    d = np.asarray(d, dtype=np.float64)
    g = np.zeros((d.shape[0], d.shape[1] + 2, d.shape[2] + 2))
    g[:, 1:-1, 1:-1] = d
    g[:, 0, 1:-1] = -d[:, 0, :]
    g[:, -1, 1:-1] = -d[:, -1, :]
    g[:, 1:-1, 0] = -d[:, :, 0]
    g[:, 1:-1, -1] = -d[:, :, -1]
    return 4.0 * d - (g[:, :-2, 1:-1] + g[:, 2:, 1:-1] + g[:, 1:-1, :-2] + g[:, 1:-1, 2:])


def loss(y: np.ndarray, target: np.ndarray, kind: str = "mse") -> float:
    """Mean over pixels of (y - t)^2 ("mse") or of (y - t) K (y - t) ("energy")."""
    d = np.asarray(y, dtype=np.float64) - target
    if kind == "energy":
        return float(np.mean(d * energy_operator(d)))
    return float(np.mean(d * d))


def loss_grad_y(y: np.ndarray, target: np.ndarray, kind: str = "mse") -> np.ndarray:
    """Derivative of `loss` with respect to y: 2 (y - t) / N, or 2 K (y - t) / N (K is
    symmetric)."""
    d = np.asarray(y, dtype=np.float64) - target
    return (2.0 / d.size) * (energy_operator(d) if kind == "energy" else d)


def backward(cache, y: np.ndarray, target: np.ndarray, kind: str = "mse"):
    """Gradient of the loss (`kind` as in `loss`) with respect to the flat weights.

    Mirrors the GPU's rounding points when the forward pass ran with bf16=True: the
    gradients entering each 32-channel convolution (dz3, dz2, and dz1) are rounded to
    bfloat16, as the GPU stores them for its matrix-core kernels."""
    rnd = bf16_round if cache["bf16"] else (lambda v: v)
    W1, W2, W3, W4 = cache["W"]
    a0, a1, a2, a3 = cache["a0"], cache["a1"], cache["a2"], cache["a3"]
    dy4 = loss_grad_y(y, target, kind)[..., None]
    dW4 = conv3x3_weight_grad(a3, dy4)
    dz3 = rnd(conv3x3_input_grad(dy4, W4) * (a3 > 0))
    dW3 = conv3x3_weight_grad(a2, dz3)
    dz2 = rnd(conv3x3_input_grad(dz3, W3) * (a2 > 0))
    dW2 = conv3x3_weight_grad(a1, dz2)
    dz1 = rnd(conv3x3_input_grad(dz2, W2) * (a1 > 0))
    dW1 = conv3x3_weight_grad(a0, dz1)
    return flatten((dW1, dW2, dW3, dW4))
