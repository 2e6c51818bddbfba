"""The learned correction network on the GPU against its CPU oracle (oracle/net.py).

Layer by layer: every layer is recomputed by the oracle from the GPU's own BF16 input
activation, so the only differences left are FP32 (GPU) against FP64 (oracle)
accumulation and, where a sum lands next to a bfloat16 rounding boundary, one
bfloat16 unit in the last place of a stored activation.  Gradients are compared with
the oracle's backward pass run on the GPU's activations; the training pairs, Adam
and the learned refinement loop against their definitions."""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_07931_amd as px
import workloads as W
from oracle import net as onet
from paper_2307_07931_amd import learned

import helpers as H

pytestmark = pytest.mark.gpu
OMEGA = 2.0 / 3.0


@pytest.fixture(scope="module")
def ctx():
    H.require_gpu()
    c = px.Context()
    yield c
    c.close()


def bf16_bits_to_f64(bits: torch.Tensor) -> np.ndarray:
    u = bits.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def activation(net, layer, B, Hh, Wd):
    out = torch.empty((B * Hh * Wd, 32), dtype=torch.int16, device="cuda")
    net.activation(layer, out)
    torch.cuda.synchronize()
    return bf16_bits_to_f64(out).reshape(B, Hh, Wd, 32)


def assert_bf16_close(gpu, ref_unrounded, abs_terms, what, max_frac=0.01):
    """gpu (BF16 values) equals the BF16 rounding of the oracle's FP64 sum except for at
    most max_frac of the elements.  Those may differ by one BF16 step plus the FP32
    accumulation bound gamma_288 * sum|terms| (abs_terms: the same convolution of the
    absolute values): the FP32 sum fell on the other side of a rounding boundary."""
    ref = onet.bf16_round(ref_unrounded)
    diff = gpu != ref
    if diff.any():
        ulp = np.abs(ref) * 2.0 ** -7
        bound = ulp + 288 * 2.0 ** -24 * abs_terms
        assert np.all(np.abs(gpu - ref)[diff] <= bound[diff] * 1.01 + 1e-30), what
        assert diff.mean() <= max_frac, (what, diff.mean())


def conv_relu(a, w):
    return np.maximum(onet.conv3x3(a, w), 0.0), onet.conv3x3(np.abs(a), np.abs(w))


@pytest.mark.parametrize("B,Hh,Wd", [(2, 37, 45), (1, 64, 96), (1, 5, 3), (3, 33, 31)])
def test_forward_layers_match_oracle(B, Hh, Wd):
    H.require_gpu()
    w = W.net_initial_weights(11)
    x = W.rng(12).standard_normal((B, Hh, Wd)) * 3.0
    net = px.Net(w)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    base = torch.full((B, Hh, Wd + 5), 7.0, dtype=torch.float32, device="cuda")
    ybig = base[:, :, :Wd]  # rows of ldy = Wd + 5
    net.forward(xd, ybig)
    torch.cuda.synchronize()
    W1, W2, W3, W4 = [onet.bf16_round(a) for a in onet.unflatten(w)]
    a0 = onet.bf16_round(x.astype(np.float32).astype(np.float64))[..., None]
    a1 = activation(net, 1, B, Hh, Wd)
    assert_bf16_close(a1, *conv_relu(a0, W1), "layer 1")
    a2 = activation(net, 2, B, Hh, Wd)
    assert_bf16_close(a2, *conv_relu(a1, W2), "layer 2")
    a3 = activation(net, 3, B, Hh, Wd)
    assert_bf16_close(a3, *conv_relu(a2, W3), "layer 3")
    ref = onet.conv3x3(a3, W4)[..., 0]
    got = ybig.cpu().numpy().astype(np.float64)
    scale = np.abs(onet.conv3x3(np.abs(a3), np.abs(W4)))[..., 0] + 1e-30
    assert np.all(np.abs(got - ref) <= 1e-5 * scale), np.max(np.abs(got - ref) / scale)
    # the padding columns of y are untouched
    assert bool((base[:, :, Wd:] == 7.0).all())
    # whole network against the oracle's own forward pass (activation flips propagate a little)
    yo, _ = onet.forward(w, x.astype(np.float32).astype(np.float64))
    assert np.linalg.norm(got - yo) <= 2e-2 * np.linalg.norm(yo)
    net.close()


@pytest.mark.parametrize("B,Hh,Wd,dt,scale", [(2, 37, 45, "f32", 1.0), (1, 64, 96, "f64", 0.37), (1, 5, 3, "f32", 1.0),
                                               (3, 33, 131, "f64", 2.5), (1, 300, 257, "f32", 1.0)])
def test_inference_equals_forward_bitwise(B, Hh, Wd, dt, scale):
    """px_net_infer (layer 1 computed inside the first convolution's patch staging) gives
    px_net_forward's output bit for bit, on ragged shapes (partial tiles in both
    directions), several images, FP64 input with a scale; and leaves no activations."""
    H.require_gpu()
    w = W.net_initial_weights(41)
    x = W.rng(42).standard_normal((B, Hh, Wd + 3)) * 2.0
    net = px.Net(w)
    xd = torch.from_numpy(x if dt == "f64" else x.astype(np.float32)).cuda()
    y1 = torch.full((B, Hh, Wd), 7.0, dtype=torch.float32, device="cuda")
    y2 = torch.full((B, Hh, Wd), -7.0, dtype=torch.float32, device="cuda")
    print(f"case: infer vs forward B={B} H={Hh} W={Wd} {dt} scale={scale}", flush=True)
    net.forward(xd[:, :, :Wd], y1, x_scale=scale)
    net.forward(xd[:, :, :Wd], y2, x_scale=scale, infer=True)
    torch.cuda.synchronize()
    assert torch.equal(y1.view(torch.int32), y2.view(torch.int32))
    out = torch.empty((B * Hh * Wd, 32), dtype=torch.int16, device="cuda")
    with pytest.raises(px.ProtoxError):
        net.activation(1, out)
    net.close()


def test_forward_fp64_input_and_scale():
    """FP64 input scaled by x_scale is rounded FP64 -> FP32 -> BF16, as the oracle's
    bf16_round of the FP64 product does."""
    H.require_gpu()
    w = W.net_initial_weights(13)
    n = 40
    r = W.rng(14).standard_normal((n, n + 24))
    net = px.Net(w)
    y = torch.empty((n, n), dtype=torch.float32, device="cuda")
    rd = torch.from_numpy(r).cuda()
    net.forward(rd[:, :n], y, x_scale=0.37)  # rows of ld n + 24
    torch.cuda.synchronize()
    a1 = activation(net, 1, 1, n, n)
    W1 = onet.bf16_round(onet.unflatten(w)[0])
    a0 = onet.bf16_round(r[:, :n] * 0.37)[None, ..., None]
    assert_bf16_close(a1, *conv_relu(a0, W1), "layer 1 from FP64")
    net.close()


@pytest.mark.parametrize("kind,B,Hh,Wd", [("mse", 2, 24, 40), ("energy", 2, 24, 40), ("mse", 1, 37, 150)])
def test_gradient_matches_oracle(kind, B, Hh, Wd):
    """Weight gradients of all four layers against the oracle's backward pass on the GPU's
    own activations; the last shape has several 64-column strips, a ragged last strip and
    a ragged last group of rows in the weight-gradient work units."""
    H.require_gpu()
    w = W.net_initial_weights(15)
    x = W.rng(16).standard_normal((B, Hh, Wd))
    t = W.rng(17).standard_normal((B, Hh, Wd)) * 0.3
    net = px.Net(w)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    grad = torch.zeros(px.NET_NPARAM, dtype=torch.float32, device="cuda")
    lo = torch.zeros(1, dtype=torch.float64, device="cuda")
    code = px.LOSS_MSE if kind == "mse" else px.LOSS_ENERGY
    net.loss_grad(xd, td, loss=code, loss_out=lo, grad=grad)
    torch.cuda.synchronize()
    # oracle backward on the GPU's activations
    Ws = tuple(onet.bf16_round(a) for a in onet.unflatten(w))
    a0 = onet.bf16_round(x.astype(np.float32).astype(np.float64))[..., None]
    cache = dict(a0=a0, a1=activation(net, 1, B, Hh, Wd), a2=activation(net, 2, B, Hh, Wd),
                 a3=activation(net, 3, B, Hh, Wd), W=Ws, bf16=True)
    y = onet.conv3x3(cache["a3"], Ws[3])[..., 0]
    tq = t.astype(np.float32).astype(np.float64)
    assert lo.item() == pytest.approx(onet.loss(y, tq, kind), rel=1e-5)
    g_ref = onet.backward(cache, y, tq, kind)
    g = grad.cpu().numpy().astype(np.float64)
    off = 0
    for k, size in enumerate(onet.SIZES):
        a, b = g[off:off + size], g_ref[off:off + size]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert rel < 1e-2, (k, rel)
        assert np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)) > 0.9999, k
        off += size
    # reproducible bit for bit
    grad2 = torch.zeros_like(grad)
    net.loss_grad(xd, td, loss=code, grad=grad2)
    torch.cuda.synchronize()
    assert torch.equal(grad, grad2)
    net.close()


def test_adam_step_matches_definition():
    H.require_gpu()
    w = W.net_initial_weights(18).astype(np.float32)
    net = px.Net(w)
    x = torch.from_numpy(W.rng(19).standard_normal((1, 16, 16)).astype(np.float32)).cuda()
    t = torch.zeros_like(x)
    grad = torch.zeros(px.NET_NPARAM, dtype=torch.float32, device="cuda")
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    ref = w.copy()
    for step in (1, 2):
        net.loss_grad(x, t, grad=grad)
        net.adam(1e-3)
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
        m = np.float32(0.9) * m + np.float32(0.1) * g
        v = np.float32(0.999) * v + np.float32(0.001) * g * g
        c1 = np.float32(1) - np.float32(0.9) ** step
        c2 = np.float32(1) - np.float32(0.999) ** step
        ref = ref - np.float32(1e-3) * (m / c1) / (np.sqrt(v / c2) + np.float32(1e-8))
        got = net.get_weights()
        np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-7)
    net.set_weights(w)
    assert np.array_equal(net.get_weights(), w)
    net.close()


@pytest.mark.parametrize("kind", ["mse", "energy"])
def test_training_pair_matches_definition(ctx, kind):
    n = 50
    phi = W.uniform_phi(n, 20)
    g = H.device_grid(phi, n, "f64")
    x = torch.empty((n, n), dtype=torch.float32, device="cuda")
    t = torch.empty_like(x)
    px.make_pair(g, n, x, t, ctx, loss=px.LOSS_MSE if kind == "mse" else px.LOSS_ENERGY)
    torch.cuda.synchronize()
    s = oracle.apply_stencil(phi, n)  # S(phi), odd reflection
    e = -phi[1:n + 1, 1:n + 1]
    xr = -s / np.sqrt(np.mean(s * s))
    en = np.mean(e * onet.energy_operator(e[None])[0]) if kind == "energy" else np.mean(e * e)
    tr = e / np.sqrt(en)
    np.testing.assert_allclose(x.cpu().numpy(), xr, rtol=2e-7, atol=1e-7)
    np.testing.assert_allclose(t.cpu().numpy(), tr, rtol=2e-7, atol=1e-7)


def setup_problem(n, f):
    phi = H.device_grid(np.zeros((n + 2, n + 2)), n, "f64")
    fd = H.device_rhs(f, n, "f64")
    h = 1.0 / n
    return phi, fd, h, OMEGA * h * h / 4.0


def loop_oracle(f, n, steps, smooth):
    """The refinement loop without the network (direction r), written from its
    definition with the oracle's residual and sweeps."""
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    phi = np.zeros((n + 2, n + 2))
    for _ in range(steps):
        r = oracle.residual(phi, f, n, h)[0]
        ad = oracle.apply_stencil(np.pad(r, 1), n) / (h * h)  # L r (odd reflection)
        a = np.sum(r * r) / np.sum(r * ad)
        phi[1:n + 1, 1:n + 1] += a * r
        phi = oracle.relax(phi, f, n, h, lam, smooth)[0]
    return phi


def test_learned_loop_without_network_matches_oracle(ctx):
    n, smooth, steps = 40, 8, 12
    f = W.grf_rhs(n, 21)
    phi, fd, h, lam = setup_problem(n, f)
    st = px.solve_learned(phi, n, fd, h, lam, ctx, use_net=False, rtol=0.0, max_sweeps=smooth * steps,
                          smooth_sweeps=smooth, tblock=4, raise_on_error=False)
    assert st.status == px.ENOTCONV and st.corrections == steps and st.sweeps == smooth * steps
    ref = loop_oracle(f, n, steps, smooth)
    got = phi.cpu().numpy()[:n + 2, :n + 2]
    np.testing.assert_allclose(got[1:n + 1, 1:n + 1], ref[1:n + 1, 1:n + 1], rtol=1e-10,
                               atol=1e-12 * np.abs(ref).max())


def test_corrupted_network_falls_back_to_plain(ctx):
    """A network whose output is NaN is rejected by the judge at its first step; the
    solve then equals plain relaxation with checks every smooth_sweeps, bit for bit."""
    n, smooth = 48, 16
    f = W.grf_rhs(n, 22)
    bad = W.net_initial_weights(23)
    bad[100] = np.nan
    net = px.Net(bad)
    phi, fd, h, lam = setup_problem(n, f)
    st = px.solve_learned(phi, n, fd, h, lam, ctx, net=net, rtol=1e-5, smooth_sweeps=smooth, tblock=8)
    assert st.rejected == 1 and st.fell_back == 1 and st.corrections == 0
    assert st.discarded_sweeps == smooth  # the undone step's sweeps count as work done
    phi2, fd2, _, _ = setup_problem(n, f)
    st2 = px.solve(phi2, n, fd2, h, lam, ctx, mode=px.SOLVE_PLAIN, rtol=1e-5, check_every=smooth, tblock=8)
    assert st.sweeps - st.discarded_sweeps == st2.sweeps
    H.assert_grid_bitwise(phi.cpu().numpy(), phi2.cpu().numpy(), n)
    net.close()


def test_judge_undoes_steps_that_raise_the_residual(ctx):
    """With one smoothing sweep per step, energy-optimal steps along r raise the residual
    norm now and then; the judge undoes those, relaxes plainly for a back-off period, and
    the solve still converges with corrections left on."""
    n = 48
    f = W.grf_rhs(n, 25)
    phi, fd, h, lam = setup_problem(n, f)
    st = px.solve_learned(phi, n, fd, h, lam, ctx, use_net=0, rtol=1e-6, smooth_sweeps=1, tblock=1)
    print(f"\njudge: {st.corrections} kept, {st.rejected} undone, {st.sweeps} sweeps")
    assert st.status == px.OK and st.rel_res_max <= 1e-6
    assert st.rejected >= 1 and st.fell_back == 0 and st.corrections >= 1
    # one sweep per kept or plain step, and one per undone step (run, then discarded)
    assert st.discarded_sweeps == st.rejected
    assert st.sweeps == st.outer_steps + st.discarded_sweeps


def test_training_reduces_loss_and_trained_net_converges(ctx):
    """Pairs from plain solves of the homogeneous problem, a short training run, and the
    learned loop with the trained network reaching the tolerance, and what the network
    gains.  Training and solves are deterministic, so the sweep counts are fixed on this
    hardware (measured: 1968 sweeps with both directions, 9312 with the network's
    direction alone, 5872 without the network, 27728 plain).  Bounds: with both
    directions the trained network at least halves the sweeps of the loop without it; its
    direction alone is the worse choice (more sweeps than without the network, which is
    recorded, not hidden); the loop without the network beats plain relaxation."""
    n = 64
    fields = [W.error_field(n, W.SEED_TRAIN_BASE + s) for s in range(4)]
    X, T = learned.training_pairs(fields, ctx, snapshots=(16, 64, 256, 1024))
    assert X.shape == (16, n, n) and torch.isfinite(X).all() and torch.isfinite(T).all()
    # normalisation: unit root-mean-square
    assert torch.allclose((X.double() ** 2).mean(dim=(1, 2)).cpu(), torch.ones(16, dtype=torch.float64), rtol=1e-5)
    net = px.Net(W.net_initial_weights(24))
    log = learned.train(net, X, T, steps=300, batch=4, lr=2e-3, log_every=50)
    first, last = log[0][1], np.mean([v for _, v in log[-2:]])
    assert last < 0.5 * first, log
    f = W.grf_rhs(n, W.SEED_EVAL_BASE)
    res = {}
    for tag, use in (("net", 1), ("both", 2), ("nonet", 0)):
        phi, fd, h, lam = setup_problem(n, f)
        res[tag] = px.solve_learned(phi, n, fd, h, lam, ctx, net=net, use_net=use, rtol=1e-10, norm=1,
                                    smooth_sweeps=16, tblock=8)
        assert res[tag].rel_res_l2 <= 1e-10
    phi, fd, h, lam = setup_problem(n, f)
    plain = px.solve(phi, n, fd, h, lam, ctx, mode=px.SOLVE_PLAIN, rtol=1e-10, norm=1, check_every=16, tblock=8)
    print(f"\nlearned loop at n={n}: sweeps with the network direction {res['net'].sweeps}, with both "
          f"directions {res['both'].sweeps}, without the network {res['nonet'].sweeps}, plain {plain.sweeps}; "
          f"seconds {res['net'].seconds:.4f} / {res['both'].seconds:.4f} / {res['nonet'].seconds:.4f} / "
          f"{plain.seconds:.4f}")
    assert res["nonet"].sweeps < plain.sweeps
    assert res["both"].sweeps <= 0.5 * res["nonet"].sweeps, (res["both"].sweeps, res["nonet"].sweeps)
    assert res["net"].sweeps > res["nonet"].sweeps  # the network's direction alone loses here
    net.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("ddt", ["f64", "f32"])
def test_correction_step_matches_definition(ctx, mode, ddt):
    """The correction step against its definition (energy-optimal coefficients over the
    allowed directions) and against brute force: the energy norm of the error after the
    step is minimal among perturbed coefficients (exact error from a dense solve)."""
    from oracle import exact
    n = 21
    h = 1.0 / n
    c = 1.0 / (h * h)
    phi0 = W.uniform_phi(n, 30)
    r = W.rng(31).standard_normal((n, n))
    d = W.rng(32).standard_normal((n, n)) + 0.5 * r
    if ddt == "f32":
        d = d.astype(np.float32).astype(np.float64)
    Sr = oracle.apply_stencil(np.pad(r, 1), n)
    Sd = oracle.apply_stencil(np.pad(d, 1), n)
    rr, dr, rsr, rsd, dsd = (np.sum(r * r), np.sum(d * r), np.sum(r * Sr), np.sum(r * Sd), np.sum(d * Sd))
    if mode == 0:
        a, b = rr / (c * rsr), 0.0
    elif mode == 1:
        a, b = 0.0, dr / (c * dsd)
    else:
        a, b = np.linalg.solve(c * np.array([[rsr, rsd], [rsd, dsd]]), [rr, dr])
    g = H.device_grid(phi0, n, "f64")
    rd = torch.zeros((n, n + 3), dtype=torch.float64, device="cuda")
    rd[:, :n] = torch.from_numpy(r).cuda()
    dd = torch.zeros((n, n + 5), dtype=H.TORCH_DTYPE[ddt], device="cuda")
    dd[:, :n] = torch.from_numpy(d).cuda().to(H.TORCH_DTYPE[ddt])
    coef = torch.zeros(2, dtype=torch.float64, device="cuda")
    px.correction_step(g, n, rd[:, :n], dd[:, :n], h, ctx, mode=mode, coef=coef)
    torch.cuda.synchronize()
    ga, gb = coef.cpu().numpy()
    assert ga == pytest.approx(a, rel=1e-11, abs=1e-300) and gb == pytest.approx(b, rel=1e-11, abs=1e-300)
    got = g.cpu().numpy()[:n + 2, :n + 2]
    want = phi0.copy()
    want[1:n + 1, 1:n + 1] = (phi0[1:n + 1, 1:n + 1] + ga * r) + gb * d
    H.assert_grid_bitwise(got, want, n)
    # Galerkin minimality: E(a, b) = <e', -L e'> with e' = e - a r - b d, L e = r
    e = exact.dense_solve(r, h)
    Ld = exact.dense_laplacian(n, h)

    def energy(x, y):
        ep = (e - x * r - y * d).ravel()
        return -ep @ (Ld @ ep)
    e0 = energy(ga, gb)
    for da_, db_ in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        if mode == 0 and db_:
            continue
        if mode == 1 and da_:
            continue
        assert e0 <= energy(ga * (1 + 1e-3 * da_) + 1e-9 * da_, gb * (1 + 1e-3 * db_) + 1e-9 * db_)
