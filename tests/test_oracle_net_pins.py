"""Pins of the network oracle: convolutions against scipy's correlate2d, adjointness of
the two gradient convolutions, backpropagation against central finite differences, and
the bfloat16 rounding against torch."""
import numpy as np
import pytest
from scipy import signal

import workloads as W
from oracle import net


def test_conv3x3_matches_scipy_correlate():
    rng = W.rng(1)
    x = rng.standard_normal((2, 9, 11, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    y = net.conv3x3(x, w)
    for b in range(2):
        for co in range(4):
            ref = sum(signal.correlate2d(x[b, :, :, ci], w[co, ci], mode="same", boundary="fill")
                      for ci in range(3))
            np.testing.assert_allclose(y[b, :, :, co], ref, rtol=1e-13, atol=1e-13)


def test_gradient_convolutions_are_adjoints():
    rng = W.rng(2)
    x = rng.standard_normal((2, 7, 8, 5))
    w = rng.standard_normal((6, 5, 3, 3))
    dy = rng.standard_normal((2, 7, 8, 6))
    lhs = np.sum(net.conv3x3(x, w) * dy)
    assert np.sum(x * net.conv3x3_input_grad(dy, w)) == pytest.approx(lhs, rel=1e-12)
    assert np.sum(w * net.conv3x3_weight_grad(x, dy)) == pytest.approx(lhs, rel=1e-12)


def test_backprop_matches_finite_differences():
    wts = W.net_initial_weights(3)
    rng = W.rng(4)
    x = rng.standard_normal((2, 10, 12))
    t = rng.standard_normal((2, 10, 12))
    y, cache = net.forward(wts, x, bf16=False)
    g = net.backward(cache, y, t)
    idx = np.concatenate([rng.integers(0, 288, 6), 288 + rng.integers(0, 9216, 6),
                          288 + 9216 + rng.integers(0, 9216, 6), 288 + 2 * 9216 + rng.integers(0, 288, 6)])
    for i in idx:
        eps = 1e-6 * max(1.0, abs(wts[i]))
        wp, wm = wts.copy(), wts.copy()
        wp[i] += eps
        wm[i] -= eps
        fd = (net.loss(net.forward(wp, x, bf16=False)[0], t) - net.loss(net.forward(wm, x, bf16=False)[0], t)) / (2 * eps)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_parameter_count():
    assert net.NPARAM == 19008 and W.net_initial_weights(0).size == 19008


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.concatenate([W.rng(5).standard_normal(100000) * 37.0,
                        (np.arange(1, 500, dtype=np.uint32) << 16 | 0x8000).view(np.float32).astype(np.float64)])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(net.bf16_round(x), ref)


def test_energy_operator_eigenvalues():
    # odd reflection at cell faces: the cell-centred sine modes sin(p pi (i+1/2)/H) sin(q pi (j+1/2)/W)
    # are eigenvectors of K with eigenvalue 4 sin^2(p pi / 2H) + 4 sin^2(q pi / 2W)
    H, Wd = 9, 12
    i = (np.arange(H) + 0.5)[:, None]
    j = (np.arange(Wd) + 0.5)[None, :]
    for p, q in ((1, 1), (2, 5), (9, 12), (4, 1)):
        v = np.sin(p * np.pi * i / H) * np.sin(q * np.pi * j / Wd)
        lam = 4 * np.sin(p * np.pi / (2 * H)) ** 2 + 4 * np.sin(q * np.pi / (2 * Wd)) ** 2
        np.testing.assert_allclose(net.energy_operator(v[None])[0], lam * v, atol=1e-12)
        assert net.loss(v[None], 0 * v[None], "energy") == pytest.approx(lam * np.mean(v * v), rel=1e-12)


def test_energy_operator_is_spd_matrix():
    # brute force on a tiny image: the matrix of K is symmetric with positive eigenvalues,
    # diagonal 4 plus 1 per edge-side of the pixel
    H, Wd = 3, 4
    M = np.array([net.energy_operator(e.reshape(1, H, Wd)).ravel() for e in np.eye(H * Wd)]).T
    assert np.array_equal(M, M.T)
    assert np.linalg.eigvalsh(M).min() > 0
    assert M[0, 0] == 6.0 and M[1, 1] == 5.0 and M[5, 5] == 4.0


def test_energy_backprop_matches_finite_differences():
    wts = W.net_initial_weights(6)
    rng = W.rng(7)
    x = rng.standard_normal((1, 8, 9))
    t = rng.standard_normal((1, 8, 9))
    y, cache = net.forward(wts, x, bf16=False)
    g = net.backward(cache, y, t, "energy")
    for i in (3, 300, 5000, 9600, 15000, 18900):
        eps = 1e-6 * max(1.0, abs(wts[i]))
        wp, wm = wts.copy(), wts.copy()
        wp[i] += eps
        wm[i] -= eps
        lp = net.loss(net.forward(wp, x, bf16=False)[0], t, "energy")
        lm = net.loss(net.forward(wm, x, bf16=False)[0], t, "energy")
        assert g[i] == pytest.approx((lp - lm) / (2 * eps), rel=1e-5, abs=1e-9), i
