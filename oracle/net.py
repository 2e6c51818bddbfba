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
for finite-difference pins).  Loss: mean squared error over all output pixels.
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


def loss(y: np.ndarray, target: np.ndarray) -> float:
    return float(np.mean((y - target) ** 2))


def backward(cache, y: np.ndarray, target: np.ndarray):
    """Gradient of the mean squared error with respect to the flat weights.

    Mirrors the GPU's rounding points when the forward pass ran with bf16=True: the
    gradients entering each 32-channel convolution (dz3, dz2, and dz1) are rounded to
    bfloat16, as the GPU stores them for its matrix-core kernels."""
    rnd = bf16_round if cache["bf16"] else (lambda v: v)
    W1, W2, W3, W4 = cache["W"]
    a0, a1, a2, a3 = cache["a0"], cache["a1"], cache["a2"], cache["a3"]
    dy = (2.0 / y.size) * (y - target)
    dy4 = dy[..., None]
    dW4 = conv3x3_weight_grad(a3, dy4)
    dz3 = rnd(conv3x3_input_grad(dy4, W4) * (a3 > 0))
    dW3 = conv3x3_weight_grad(a2, dz3)
    dz2 = rnd(conv3x3_input_grad(dz3, W3) * (a2 > 0))
    dW2 = conv3x3_weight_grad(a1, dz2)
    dz1 = rnd(conv3x3_input_grad(dz2, W2) * (a1 > 0))
    dW1 = conv3x3_weight_grad(a0, dz1)
    return flatten((dW1, dW2, dW3, dW4))
