"""The network's kernels at a real size: a 1024 x 1024 image has 4096 tiles of the
matrix-core convolution, twice the 2048 blocks it launches, so every block runs its tile
loop (with the next tile's patch loads in flight) and every tile is compared; the
weight-gradient kernels run their full work-unit grids.

Bars, element by element:
* forward activations: the BF16 rounding of the oracle's FP64 convolution of the GPU's
  own input activation, except where the FP32 sum lies within its accumulation bound
  (gamma_288 times the sum of |terms|) of a BF16 rounding boundary: there one BF16 step;
* the FP32 output of layer 4: within gamma_288 of the sum of |terms|;
* weight gradients: the oracle's backward pass on the GPU's activations, within a bound
  propagated layer by layer: each gradient entering a 32-channel convolution is stored
  in BF16 by both sides (one rounding each, at most 2^-8 relative), the difference of the
  upstream gradients passes through |W|, and the weight gradient's FP32 sums add at most
  gamma_D of the sum of |products| (D = 2048 additions per sum at this size: 64
  matrix-core steps of 16 products per work unit, then 32 + 32 partial sums; the thin
  layers' lanes add 128 products, then 64 + 64 partials)."""
import numpy as np
import pytest
import torch

import paper_2307_07931_amd as px
import workloads as W
from oracle import net as onet

import helpers as H
from test_gpu_net import activation, assert_bf16_close, conv_relu

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24
N = 1024


def gamma32(d):
    return d * U32 / (1 - d * U32)


def test_forward_1024_every_tile_matches_oracle():
    H.require_gpu()
    w = W.net_initial_weights(31)
    x = W.rng(32).standard_normal((1, N, N)) * 2.0
    net = px.Net(w)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    y = torch.empty_like(xd)
    print(f"case: net forward 1x{N}x{N}", flush=True)
    net.forward(xd, y)
    torch.cuda.synchronize()
    W1, W2, W3, W4 = [onet.bf16_round(a) for a in onet.unflatten(w)]
    a0 = onet.bf16_round(x.astype(np.float32).astype(np.float64))[..., None]
    a1 = activation(net, 1, 1, N, N)
    assert_bf16_close(a1, *conv_relu(a0, W1), "layer 1")
    a2 = activation(net, 2, 1, N, N)
    assert_bf16_close(a2, *conv_relu(a1, W2), "layer 2")
    a3 = activation(net, 3, 1, N, N)
    assert_bf16_close(a3, *conv_relu(a2, W3), "layer 3")
    ref = onet.conv3x3(a3, W4)[..., 0]
    mag = onet.conv3x3(np.abs(a3), np.abs(W4))[..., 0]
    got = y.cpu().numpy().astype(np.float64)[0]
    assert np.all(np.abs(got - ref[0]) <= gamma32(288) * mag[0] + 1e-30)
    # inference (layers 1 and 2 fused, every block looping over its tiles) gives the same bits
    y2 = torch.empty_like(y)
    net.forward(xd, y2, infer=True)
    torch.cuda.synchronize()
    assert torch.equal(y.view(torch.int32), y2.view(torch.int32))
    net.close()


def abs_k(v):
    """|K| applied to v >= 0: 4 v + the four neighbours' v, a neighbour outside the image
    standing for the pixel itself (odd reflection: -d has the same magnitude)."""
    p = np.pad(v, ((0, 0), (1, 1), (1, 1)), mode="edge")
    return 4 * v + p[:, :-2, 1:-1] + p[:, 2:, 1:-1] + p[:, 1:-1, :-2] + p[:, 1:-1, 2:]


def weight_grad_abs(act, e):
    return np.abs(onet.conv3x3_weight_grad(np.abs(act), np.abs(e)))


@pytest.mark.parametrize("kind", ["mse", "energy"])
def test_gradient_1024_elementwise_within_propagated_bound(kind):
    H.require_gpu()
    w = W.net_initial_weights(33)
    x = W.rng(34).standard_normal((1, N, N))
    t = W.rng(35).standard_normal((1, N, N)) * 0.3
    net = px.Net(w)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    grad = torch.zeros(px.NET_NPARAM, dtype=torch.float32, device="cuda")
    print(f"case: net gradient ({kind}) 1x{N}x{N}", flush=True)
    net.loss_grad(xd, td, loss=px.LOSS_MSE if kind == "mse" else px.LOSS_ENERGY, grad=grad)
    torch.cuda.synchronize()
    Ws = tuple(onet.bf16_round(a) for a in onet.unflatten(w))
    W1, W2, W3, W4 = Ws
    a0 = onet.bf16_round(x.astype(np.float32).astype(np.float64))[..., None]
    a1, a2, a3 = (activation(net, k, 1, N, N) for k in (1, 2, 3))
    cache = dict(a0=a0, a1=a1, a2=a2, a3=a3, W=Ws, bf16=True)
    y = onet.conv3x3(a3, W4)[..., 0]
    tq = t.astype(np.float32).astype(np.float64)
    g_ref = onet.backward(cache, y, tq, kind)
    g = grad.cpu().numpy().astype(np.float64)
    # error of the GPU's dy = dloss/dy: its y is an FP32 sum of 288 terms (within gamma_288 of
    # the sum of |terms| of the oracle's), then y - t and (energy) K d = 4 d - (neighbours) in
    # FP32, times 2 / N (a power of two)
    npix = N * N
    delta_y = gamma32(288) * onet.conv3x3(np.abs(a3), np.abs(W4))[..., 0]
    d = np.abs(y - tq)
    if kind == "mse":
        ey = 2.0 / npix * (delta_y + gamma32(2) * d)
    else:
        ey = 2.0 / npix * (abs_k(delta_y) + gamma32(8) * abs_k(d))
    dz = onet.loss_grad_y(y, tq, kind)[..., None]
    e = ey[..., None]
    bounds = []
    layers = ((W4, a3), (W3, a2), (W2, a1), (W1, a0))
    for li, (Wl, act_in) in enumerate(layers):
        # this layer's weight gradient sums dz * act_in over the pixels: the difference of
        # dz passes through |act_in|, and the FP32 sums add gamma_D of the |products|
        bounds.append(weight_grad_abs(act_in, e) + gamma32(2048) * weight_grad_abs(act_in, np.abs(dz) + e))
        if li == len(layers) - 1:
            break
        # the gradient entering the layer below: input_grad(dz, W) * (act_in > 0), an FP32
        # sum of at most 288 terms on the GPU, then stored in BF16 by both sides (each
        # rounding moves a value by at most 2^-8 of it)
        mask = act_in > 0
        pre = onet.conv3x3_input_grad(dz, Wl) * mask
        e_pre = (onet.conv3x3_input_grad(e, np.abs(Wl)) + gamma32(288) * onet.conv3x3_input_grad(np.abs(dz), np.abs(Wl))) * mask
        dz = onet.bf16_round(pre)
        e = e_pre * (1 + 2.0 ** -8) + 2.0 ** -7 * 1.01 * np.abs(dz)
    # bounds are in layer order 4, 3, 2, 1; flatten as the oracle does (1, 2, 3, 4)
    b_flat = np.concatenate([bounds[3].ravel(), bounds[2].ravel(), bounds[1].ravel(), bounds[0].ravel()])
    assert b_flat.shape == g.shape
    bad = np.abs(g - g_ref) > b_flat * 1.001 + 1e-30
    assert not bad.any(), (int(bad.sum()), np.flatnonzero(bad)[:5])
    # and the bound is informative: well below the magnitude of the gradients it bounds
    rel = np.linalg.norm(b_flat) / np.linalg.norm(g_ref)
    print(f"\n{kind}: elementwise bound / |g| = {rel:.3g}; max |g - g_ref| / bound = "
          f"{np.max(np.abs(g - g_ref) / (b_flat + 1e-30)):.3g}")
    net.close()
