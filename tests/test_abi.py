"""The C ABI on the CPU: the library loads, exports every declared symbol, and
rejects bad arguments on the host before any HIP call (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2307_07931_amd as px

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "protox.h")

FAKE = 0x10000  # an aligned, never-dereferenced address: validation fails before use
FAKE2 = 0x20000000


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(px_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = px.lib()
    names = declared_functions()
    assert len(names) >= 10
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(px.EXPORTS) <= set(names)


def test_version_and_empty_error():
    assert "gfx950" in px.version()


@pytest.fixture
def ctx():
    h = ctypes.c_void_p()
    assert px.lib().px_ctx_create(0, ctypes.byref(h)) == px.OK  # allocates nothing
    yield h
    assert px.lib().px_ctx_destroy(h) == px.OK


def relax(handle, **kw):
    a = dict(phi_in=FAKE, phi_out=FAKE2, n=64, ld=66, dtype=px.F64, f=FAKE2 * 2, ld_f=64,
             h=1 / 64, lam=1e-5, nsweeps=10, tblock=1, bc=0, resmode=2, norms=FAKE2 * 3, ctx=handle)
    a.update(kw)
    P = ctypes.c_void_p
    return px.lib().px_relax_fused(P(a["phi_in"]), P(a["phi_out"]), a["n"], a["ld"], a["dtype"],
                                   P(a["f"]), a["ld_f"], a["h"], a["lam"], a["nsweeps"], a["tblock"],
                                   a["bc"], a["resmode"], P(a["norms"]), a["ctx"], None)


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), px.EINVAL),
    (dict(n=-3), px.EINVAL),
    (dict(ld=65), px.EINVAL),
    (dict(ld_f=63), px.EINVAL),
    (dict(phi_in=0), px.EINVAL),
    (dict(phi_out=0), px.EINVAL),
    (dict(f=0), px.EINVAL),
    (dict(phi_in=FAKE + 4), px.EINVAL),       # misaligned for FP64
    (dict(dtype=7), px.EINVAL),
    (dict(bc=5), px.EINVAL),
    (dict(resmode=3), px.EINVAL),
    (dict(norms=0), px.EINVAL),
    (dict(norms=FAKE2 * 3 + 4), px.EINVAL),
    (dict(h=0.0), px.EINVAL),
    (dict(h=float("nan")), px.EINVAL),
    (dict(lam=-1.0), px.EINVAL),
    (dict(lam=float("inf")), px.EINVAL),
    (dict(nsweeps=-1), px.EINVAL),
    (dict(tblock=9), px.EINVAL),
    (dict(tblock=-1), px.EINVAL),
    (dict(ctx=None), px.EINVAL),
    (dict(phi_out=FAKE + 8 * 100), px.EALIAS),  # overlaps phi_in
    (dict(f=FAKE2 + 8 * 66), px.EALIAS),        # overlaps phi_out
])
def test_relax_validation(ctx, kw, code):
    assert relax(ctx, **kw) == code
    assert px.last_error() != ""


def relax_noalloc(**kw):
    a = dict(phi_in=FAKE, phi_out=FAKE2, n=64, ld=66, dtype=px.F64, f=FAKE2 * 2, ld_f=64,
             h=1 / 64, lam=1e-5, nsweeps=8, bc=0, resmode=2, norms=FAKE2 * 3)
    a.update(kw)
    P = ctypes.c_void_p
    return px.lib().px_relax_fused_noalloc(P(a["phi_in"]), P(a["phi_out"]), a["n"], a["ld"], a["dtype"],
                                           P(a["f"]), a["ld_f"], a["h"], a["lam"], a["nsweeps"], a["bc"],
                                           a["resmode"], P(a["norms"]), None)


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), px.EINVAL),
    (dict(ld=65), px.EINVAL),
    (dict(phi_in=0), px.EINVAL),
    (dict(f=0), px.EINVAL),
    (dict(dtype=7), px.EINVAL),
    (dict(bc=5), px.EINVAL),
    (dict(resmode=3), px.EINVAL),
    (dict(norms=0), px.EINVAL),
    (dict(h=0.0), px.EINVAL),
    (dict(lam=float("nan")), px.EINVAL),
    (dict(nsweeps=0), px.EINVAL),   # one launch of 1..8 sweeps only
    (dict(nsweeps=9), px.EINVAL),
    (dict(phi_out=FAKE + 8 * 100), px.EALIAS),
    (dict(f=FAKE2 + 8 * 66), px.EALIAS),
    # more reduction partials than the fixed array holds (rejected before any HIP call)
    (dict(n=40000, ld=40002, phi_out=1 << 40, f=2 << 40, ld_f=40000, norms=3 << 40), px.EINVAL),
])
def test_relax_noalloc_validation(kw, code):
    assert relax_noalloc(**kw) == code
    assert px.last_error() != ""


def test_relax_noalloc_fits_every_grid_up_to_16384():
    """The fixed partials array holds the wave tiles of every default launch up to n = 16384
    (the limit the header states), for every precision, sweep count and residual mode."""
    from paper_2307_07931_amd import build  # noqa: F401  (the library is built)
    cap = 1 << 17
    for dtype, V in ((px.F64, 2), (px.F32, 4), (px.BF16, 4)):
        for k in range(1, 9):
            for rm in (1, 2):
                nl = k + (1 if rm == 2 else 0)
                rows = default_rows(dtype, 16384, k)
                halo = 0 if nl == 1 else (nl + V - 1) // V * V
                stride = 64 * V - 2 * halo
                tiles = -(-(16384 + 2) // stride) * -(-(16384 + 2) // rows)
                assert tiles <= cap, (dtype, k, rm, tiles)


def default_rows(dtype, n, sweeps):
    """The library's default tile height (relax_default_rows), restated."""
    if dtype == px.F64:
        rows = 48 if sweeps <= 2 else (38 if sweeps <= 6 else 32)
    else:
        rows = 20 if sweeps <= 7 else 32
    rows = min(rows, max(8, (n + 2) // 16))
    if (sweeps + 1) % 3 == 0:
        u = sweeps + 1
        rows -= (rows + 2 * sweeps) % u
        if rows < 8:
            rows += u
    return rows


def test_relax_bf16_alignment_is_two_bytes(ctx):
    # 2-byte alignment is enough for BF16; odd address is not
    assert relax(ctx, dtype=px.BF16, phi_in=FAKE + 1) == px.EINVAL


def test_stencil_validation():
    P = ctypes.c_void_p
    t = (ctypes.c_double * 9)(*px.LAPLACE_TAPS)
    L = px.lib()
    assert L.px_apply_stencil(P(FAKE), 8, 10, 0, P(FAKE2), 8, None, 1.0, 0, None) == px.EINVAL
    assert L.px_apply_stencil(P(FAKE), 8, 9, 0, P(FAKE2), 8, t, 1.0, 0, None) == px.EINVAL
    assert L.px_apply_stencil(P(FAKE), 8, 10, 0, P(FAKE + 80), 8, t, 1.0, 0, None) == px.EALIAS
    bad = (ctypes.c_double * 9)(*([float("nan")] + [0.0] * 8))
    assert L.px_apply_stencil(P(FAKE), 8, 10, 0, P(FAKE2), 8, bad, 1.0, 0, None) == px.EINVAL
    assert L.px_apply_stencil(P(FAKE), 8, 10, 0, P(FAKE2), 8, t, float("inf"), 0, None) == px.EINVAL


def test_residual_and_jacobi_validation(ctx):
    P = ctypes.c_void_p
    L = px.lib()
    assert L.px_residual(P(FAKE), 8, 10, 0, P(FAKE2), 8, 0.125, 0, None, 0, None, ctx, None) == px.EINVAL
    assert L.px_residual(P(FAKE), 8, 10, 0, P(FAKE2), 8, 0.125, 0, None, 0, P(FAKE2 * 2), None,
                         None) == px.EINVAL
    assert L.px_residual(P(FAKE), 8, 10, 0, P(FAKE2), 8, 0.125, 0, P(FAKE2 + 8), 8, P(FAKE2 * 2),
                         ctx, None) == px.EALIAS
    assert L.px_jacobi_update(P(FAKE), 8, 10, 0, P(FAKE2), 8, P(FAKE2 * 2), 8, 0.125, 0.0,
                              None) == px.EINVAL
    assert L.px_jacobi_update(P(FAKE), 8, 10, 0, P(FAKE + 16), 8, P(FAKE2 * 2), 8, 0.125, 1e-3,
                              None) == px.EALIAS


def test_solve_validation(ctx):
    P = ctypes.c_void_p
    L = px.lib()
    st = px._SolveStats()

    def solve(dtype=0, **kw):
        o = px._SolveOpts(kw.get("mode", 0), kw.get("norm", 0), kw.get("rtol", 1e-8),
                          kw.get("max_sweeps", 100), 10, 8, kw.get("tblock", 0), kw.get("bc", 0))
        return L.px_solve(P(FAKE), 8, 10, dtype, P(FAKE2), 8, 0.125, 1e-3, ctypes.byref(o),
                          ctypes.byref(st), ctx, None)

    assert solve(mode=9) == px.EINVAL
    assert solve(mode=px.SOLVE_MIXED_F32, dtype=px.F32) == px.EINVAL
    assert solve(rtol=-1.0) == px.EINVAL
    assert solve(norm=2) == px.EINVAL
    assert solve(max_sweeps=-5) == px.EINVAL
    assert solve(tblock=12) == px.EINVAL
    assert solve(bc=3) == px.EINVAL
    assert solve(bc=px.BC_PERIODIC, mode=px.SOLVE_MIXED_F32) == px.EUNSUPPORTED
    assert L.px_solve(P(FAKE), 8, 10, 0, P(FAKE2), 8, 0.125, 1e-3, None, ctypes.byref(st), ctx,
                      None) == px.EINVAL


def test_autotune_validation(ctx):
    P = ctypes.c_void_p
    L = px.lib()
    assert L.px_autotune(P(FAKE), P(FAKE2), 0, 66, 0, P(FAKE2 * 2), 64, 0, ctx, None, None, None,
                         None) == px.EINVAL
    assert L.px_autotune(P(FAKE), P(FAKE + 8), 64, 66, 0, P(FAKE2 * 2), 64, 0, ctx, None, None, None,
                         None) == px.EALIAS
    assert L.px_autotune(P(FAKE), P(FAKE2), 64, 66, 0, P(FAKE2 * 2), 64, 9, ctx, None, None, None,
                         None) == px.EINVAL
    assert L.px_autotune(P(FAKE), P(FAKE2), 64, 66, 0, P(FAKE2 * 2), 64, 0, None, None, None, None,
                         None) == px.EINVAL


def test_ctx_validation():
    L = px.lib()
    h = ctypes.c_void_p()
    assert L.px_ctx_create(-1, ctypes.byref(h)) == px.EINVAL
    assert L.px_ctx_create(0, None) == px.EINVAL
    assert L.px_ctx_destroy(None) == px.OK
    assert L.px_ctx_set_tile_rows(None, 4) == px.EINVAL
    assert L.px_ctx_reserve(None, 8, 10, 0) == px.EINVAL


def test_python_binding_rejects_bad_layouts():
    torch = pytest.importorskip("torch")
    phi = torch.zeros(10, 10, dtype=torch.float64)
    with pytest.raises(ValueError):
        px._ld(phi.t(), 10, 10, "phi")  # not unit column stride
    with pytest.raises(ValueError):
        px._ld(phi, 9, 10, "phi")
    with pytest.raises(TypeError):
        px.dtype_code(torch.zeros(1, dtype=torch.int32))


def test_batched_validation(ctx):
    L = px.lib()
    P = ctypes.c_void_p
    probs = (px._Problem * 2)(px._Problem(FAKE, FAKE2, 8, 16, 8, 0.125, 1e-3),
                              px._Problem(FAKE2 * 2, FAKE2 * 3, 8, 16, 8, 0.125, 1e-3))
    ok = dict(nprob=2, dtype=px.F64, nsweeps=4, tblock=2, bc=0, resmode=0)

    def relax(**kw):
        a = dict(ok)
        a.update(kw)
        return L.px_relax_batched(kw.get("probs", probs), a["nprob"], a["dtype"], a["nsweeps"], a["tblock"],
                                  a["bc"], a["resmode"], None, ctx, None)

    assert relax(nprob=0) == px.EINVAL
    assert relax(nsweeps=0) == px.EINVAL
    assert relax(tblock=9) == px.EINVAL
    assert relax(resmode=2) == px.EINVAL            # FINAL needs norms
    assert relax(resmode=1) == px.EUNSUPPORTED      # lagged norms are not reported for batches
    assert relax(bc=px.BC_PERIODIC) == px.EUNSUPPORTED
    assert relax(bc=3) == px.EINVAL
    bad = (px._Problem * 2)(probs[0], px._Problem(FAKE + 8, FAKE2 * 3, 8, 16, 8, 0.125, 1e-3))
    assert relax(probs=bad) == px.EINVAL           # not 16-byte aligned
    over = (px._Problem * 2)(probs[0], px._Problem(FAKE + 256, FAKE2 * 3, 8, 16, 8, 0.125, 1e-3))
    assert relax(probs=over) == px.EALIAS          # two problems share memory
    oddld = (px._Problem * 1)(px._Problem(FAKE, FAKE2, 8, 11, 8, 0.125, 1e-3))
    assert relax(probs=oddld, nprob=1) == px.EINVAL
    st = (px._SolveStats * 2)()
    o = px._SolveOpts(px.SOLVE_PLAIN, 0, 1e-8, 100, 0, 8, 0, 0)
    assert L.px_solve_batched(probs, 2, ctypes.byref(o), st, ctx, None) == px.EUNSUPPORTED
    o = px._SolveOpts(px.SOLVE_MIXED_F32, 3, 1e-8, 100, 0, 8, 0, 0)
    assert L.px_solve_batched(probs, 2, ctypes.byref(o), st, ctx, None) == px.EINVAL
    assert L.px_solve_batched(probs, 2, None, st, ctx, None) == px.EINVAL
    k = ctypes.c_int()
    assert L.px_autotune_batched(probs, 0, px.F64, 0, ctx, None, ctypes.byref(k)) == px.EINVAL
    assert L.px_autotune_batched(probs, 2, 7, 0, ctx, None, ctypes.byref(k)) == px.EINVAL
    assert L.px_autotune_batched(probs, 2, px.F64, 5, ctx, None, ctypes.byref(k)) == px.EINVAL
    assert L.px_autotune_batched(probs, 2, px.F64, 0, None, None, ctypes.byref(k)) == px.EINVAL
    assert L.px_autotune_batched(over, 2, px.F64, 0, ctx, None, ctypes.byref(k)) == px.EALIAS


def test_net_validation(ctx):
    L = px.lib()
    P = ctypes.c_void_p
    h = ctypes.c_void_p()
    assert L.px_net_create(0, None, ctypes.byref(h)) == px.EINVAL
    assert "NULL" in px.last_error()
    w = (ctypes.c_float * px.NET_NPARAM)()
    assert L.px_net_create(0, w, None) == px.EINVAL
    assert L.px_net_destroy(None) == px.OK
    assert L.px_net_set_weights(None, w) == px.EINVAL
    assert L.px_net_get_weights(None, w) == px.EINVAL
    assert L.px_net_forward(None, P(FAKE), px.F32, 8, 1, 8, 8, 1.0, P(FAKE2), 8, None) == px.EINVAL
    assert L.px_net_loss_grad(None, P(FAKE), P(FAKE2), 1, 8, 8, 0, None, None, None) == px.EINVAL
    assert L.px_net_adam(None, ctypes.c_float(1e-3), None) == px.EINVAL
    assert L.px_net_activation(None, 1, P(FAKE), None) == px.EINVAL
    # training pairs: size, pointers, loss kind, overlap
    mk = lambda **kw: L.px_net_make_pair(P(kw.get("phi", FAKE)), kw.get("n", 64), kw.get("ld", 66),
                                         kw.get("loss", 0), P(kw.get("x", FAKE2)), P(kw.get("t", FAKE2 * 2)),
                                         ctx, None)
    assert mk(n=0) == px.EINVAL
    assert mk(ld=65) == px.EINVAL
    assert mk(phi=0) == px.EINVAL
    assert mk(x=0) == px.EINVAL
    assert mk(loss=7) == px.EINVAL
    assert mk(x=FAKE + 8) == px.EALIAS
    assert mk(t=FAKE2 + 64) == px.EALIAS


def test_solve_learned_validation(ctx):
    L = px.lib()
    P = ctypes.c_void_p

    def run(opts=True, net=None, **kw):
        o = px._LearnedOpts(kw.get("norm", 0), kw.get("rtol", 1e-10), kw.get("max_sweeps", 100),
                            kw.get("smooth", 16), kw.get("tblock", 0), kw.get("use_net", 0), kw.get("judge", 2))
        return L.px_solve_learned(P(kw.get("phi", FAKE)), kw.get("n", 64), kw.get("ld", 66),
                                  P(kw.get("f", FAKE2)), kw.get("ld_f", 64), kw.get("h", 1 / 64),
                                  kw.get("lam", 1e-5), net, ctypes.byref(o) if opts else None, None,
                                  kw.get("ctx", ctx), None)

    assert run(opts=False) == px.EINVAL
    assert run(ctx=None) == px.EINVAL
    assert run(n=0) == px.EINVAL
    assert run(phi=0) == px.EINVAL
    assert run(f=0) == px.EINVAL
    assert run(h=0.0) == px.EINVAL
    assert run(lam=-1.0) == px.EINVAL
    assert run(rtol=float("nan")) == px.EINVAL
    assert run(norm=2) == px.EINVAL
    assert run(max_sweeps=-1) == px.EINVAL
    assert run(smooth=0) == px.EINVAL
    assert run(tblock=9) == px.EINVAL
    assert run(use_net=3) == px.EINVAL
    assert run(judge=3) == px.EINVAL
    assert run(use_net=-1) == px.EINVAL
    assert run(use_net=1) == px.EINVAL  # no network
    assert "network" in px.last_error()
    assert run(f=FAKE + 8) == px.EALIAS


def test_correction_step_validation(ctx):
    L = px.lib()
    P = ctypes.c_void_p

    def run(**kw):
        return L.px_correction_step(P(kw.get("phi", FAKE)), kw.get("n", 64), kw.get("ld", 66), P(kw.get("r", FAKE2)),
                                    kw.get("ld_r", 64), P(kw.get("d", FAKE2 * 2)), kw.get("ddt", px.F32),
                                    kw.get("ld_d", 64), kw.get("h", 1 / 64), kw.get("mode", 2), None,
                                    kw.get("ctx", ctx), None)

    assert run(ctx=None) == px.EINVAL
    assert run(n=0) == px.EINVAL
    assert run(ld=65) == px.EINVAL
    assert run(phi=0) == px.EINVAL
    assert run(r=0) == px.EINVAL
    assert run(ld_r=63) == px.EINVAL
    assert run(mode=3) == px.EINVAL
    assert run(d=0) == px.EINVAL  # mode 2 needs d
    assert run(ddt=px.BF16) == px.EINVAL
    assert run(ld_d=10) == px.EINVAL
    assert run(h=0.0) == px.EINVAL
    assert run(r=FAKE + 64) == px.EALIAS
    assert run(d=FAKE + 64) == px.EALIAS


def test_relax_boxes_validation(ctx):
    """px_relax_boxes checks the layout, equal box sizes and the exchange period on the host."""
    P = ctypes.c_void_p
    L = px.lib()
    arr = (px._Problem * 2)()
    arr[0] = px._Problem(FAKE, FAKE2, 16, 18, 16, 1 / 32, 1e-5)
    arr[1] = px._Problem(FAKE * 64, FAKE2 * 4, 16, 18, 16, 1 / 32, 1e-5)
    assert L.px_relax_boxes(arr, 0, 2, px.F64, 4, 1, 0, ctx, None) == px.EINVAL      # layout
    assert L.px_relax_boxes(arr, 2, 1, px.F64, 4, 3, 0, ctx, None) == px.EINVAL      # 4 % 3 != 0
    assert L.px_relax_boxes(arr, 2, 1, px.F64, 4, 9, 0, ctx, None) == px.EINVAL      # exchange > 8
    assert L.px_relax_boxes(arr, 2, 1, px.F64, 4, 1, 7, ctx, None) == px.EINVAL      # bc
    arr[1] = px._Problem(FAKE * 64, FAKE2 * 4, 20, 22, 20, 1 / 32, 1e-5)
    assert L.px_relax_boxes(arr, 2, 1, px.F64, 4, 1, 0, ctx, None) == px.EINVAL      # unequal n
    assert "same n" in px.last_error()
