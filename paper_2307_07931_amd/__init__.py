"""Python binding of the MI355X fused Poisson relaxation library (libprotox.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/protox.h``.  PyTorch provides
device memory and streams.  If the shared library has not been built the
import of any function fails loudly -- there is no CPU fallback.

Layout conventions (Section IV of the ProtoX paper: an n x n box of cells with
one ghost layer, m = n + 2):

* ``phi``: 2-D tensor of shape (n+2, ld'), unit column stride, row stride ld
  (ld >= n+2); interior at [1:n+1, 1:n+1].
* ``f``: 2-D tensor of shape (n, >= n), unit column stride, row stride ld_f.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprotox.so")

# px_status
OK, EINVAL, EUNSUPPORTED, EALIAS, EHIP, ENOTCONV, EDIVERGED, ENONFINITE, ENOMEM = 0, -1, -2, -3, -4, -5, -6, -7, -8
STATUS_NAMES = {0: "PX_OK", -1: "PX_EINVAL", -2: "PX_EUNSUPPORTED", -3: "PX_EALIAS", -4: "PX_EHIP",
                -5: "PX_ENOTCONV", -6: "PX_EDIVERGED", -7: "PX_ENONFINITE", -8: "PX_ENOMEM"}
F64, F32, BF16 = 0, 1, 2
BC_DIRICHLET0, BC_GHOST_FIXED, BC_PERIODIC = 0, 1, 2
RES_NONE, RES_LAGGED, RES_FINAL = 0, 1, 2
SOLVE_PLAIN, SOLVE_MIXED_F32, SOLVE_MIXED_BF16 = 0, 1, 2
LAPLACE_TAPS = (0.0, 1.0, 0.0, 1.0, -4.0, 1.0, 0.0, 1.0, 0.0)

_DTYPE_CODE = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}


class ProtoxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class _SolveOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("norm", ctypes.c_int), ("rtol", ctypes.c_double),
                ("max_sweeps", ctypes.c_int64), ("check_every", ctypes.c_int),
                ("inner_sweeps", ctypes.c_int), ("tblock", ctypes.c_int), ("bc", ctypes.c_int)]


class _SolveStats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("outer_steps", ctypes.c_int64),
                ("res_max", ctypes.c_double), ("res_l2", ctypes.c_double),
                ("rel_res_max", ctypes.c_double), ("rel_res_l2", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class _LearnedOpts(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_int), ("rtol", ctypes.c_double), ("max_sweeps", ctypes.c_int64),
                ("smooth_sweeps", ctypes.c_int), ("tblock", ctypes.c_int), ("use_net", ctypes.c_int),
                ("judge", ctypes.c_int)]


class _LearnedStats(ctypes.Structure):
    _fields_ = [("base", _SolveStats), ("corrections", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("fell_back", ctypes.c_int), ("discarded_sweeps", ctypes.c_int64)]


class _Problem(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_void_p), ("f", ctypes.c_void_p), ("n", ctypes.c_int),
                ("ld", ctypes.c_int), ("ld_f", ctypes.c_int), ("h", ctypes.c_double),
                ("lambda_", ctypes.c_double)]


EXPORTS = ("px_ctx_create", "px_ctx_destroy", "px_ctx_reserve", "px_ctx_set_tile_rows",
           "px_autotune", "px_last_error", "px_version", "px_apply_stencil", "px_residual",
           "px_jacobi_update", "px_relax_fused", "px_solve", "px_relax_batched", "px_solve_batched",
           "px_autotune_batched", "px_net_create", "px_net_destroy", "px_net_set_weights", "px_net_get_weights",
           "px_net_forward", "px_net_loss_grad", "px_net_adam", "px_net_activation",
           "px_net_make_pair", "px_correction_step", "px_solve_learned", "px_relax_fused_noalloc",
           "px_net_infer", "px_relax_boxes")

_lib = None


def lib() -> ctypes.CDLL:
    """Load libprotox.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2307_07931_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.px_ctx_create.argtypes = [I, ctypes.POINTER(P)]
    L.px_ctx_destroy.argtypes = [P]
    L.px_ctx_reserve.argtypes = [P, I, I, I]
    L.px_ctx_set_tile_rows.argtypes = [P, I]
    L.px_last_error.restype = ctypes.c_char_p
    L.px_last_error.argtypes = []
    L.px_version.restype = ctypes.c_char_p
    L.px_version.argtypes = []
    L.px_apply_stencil.argtypes = [P, I, I, I, P, I, ctypes.POINTER(D), D, I, P]
    L.px_residual.argtypes = [P, I, I, I, P, I, D, I, P, I, P, P, P]
    L.px_jacobi_update.argtypes = [P, I, I, I, P, I, P, I, D, D, P]
    L.px_relax_fused.argtypes = [P, P, I, I, I, P, I, D, D, I, I, I, I, P, P, P]
    L.px_relax_fused_noalloc.argtypes = [P, P, I, I, I, P, I, D, D, I, I, I, P, P]
    L.px_solve.argtypes = [P, I, I, I, P, I, D, D, ctypes.POINTER(_SolveOpts),
                           ctypes.POINTER(_SolveStats), P, P]
    L.px_autotune.argtypes = [P, P, I, I, I, P, I, I, P, P, ctypes.POINTER(I), ctypes.POINTER(I),
                              ctypes.POINTER(D)]
    L.px_relax_batched.argtypes = [ctypes.POINTER(_Problem), I, I, I, I, I, I, P, P, P]
    L.px_relax_boxes.argtypes = [ctypes.POINTER(_Problem), I, I, I, I, I, I, P, P]
    L.px_autotune_batched.argtypes = [ctypes.POINTER(_Problem), I, I, I, P, P, ctypes.POINTER(I)]
    L.px_solve_batched.argtypes = [ctypes.POINTER(_Problem), I, ctypes.POINTER(_SolveOpts),
                                   ctypes.POINTER(_SolveStats), P, P]
    F = ctypes.POINTER(ctypes.c_float)
    L.px_net_create.argtypes = [I, F, ctypes.POINTER(P)]
    L.px_net_destroy.argtypes = [P]
    L.px_net_set_weights.argtypes = [P, F]
    L.px_net_get_weights.argtypes = [P, F]
    L.px_net_forward.argtypes = [P, P, I, I, I, I, I, D, P, I, P]
    L.px_net_infer.argtypes = [P, P, I, I, I, I, I, D, P, I, P]
    L.px_net_loss_grad.argtypes = [P, P, P, I, I, I, I, P, P, P]
    L.px_net_adam.argtypes = [P, ctypes.c_float, P]
    L.px_net_activation.argtypes = [P, I, P, P]
    L.px_net_make_pair.argtypes = [P, I, I, I, P, P, P, P]
    L.px_correction_step.argtypes = [P, I, I, P, I, P, I, I, D, I, P, P, P]
    L.px_solve_learned.argtypes = [P, I, I, P, I, D, D, P, ctypes.POINTER(_LearnedOpts),
                                   ctypes.POINTER(_LearnedStats), P, P]
    for nm in ("px_autotune_batched", "px_net_create", "px_net_destroy", "px_net_set_weights", "px_net_get_weights",
               "px_net_forward", "px_net_infer", "px_net_loss_grad", "px_net_adam", "px_net_activation",
               "px_net_make_pair", "px_correction_step", "px_solve_learned",
               "px_relax_batched", "px_relax_boxes", "px_solve_batched", "px_ctx_create", "px_ctx_destroy",
               "px_ctx_reserve", "px_ctx_set_tile_rows", "px_autotune",
               "px_apply_stencil", "px_residual", "px_jacobi_update", "px_relax_fused", "px_solve"):
        getattr(L, nm).restype = I
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        raise ProtoxError(status, lib().px_last_error().decode())


def last_error() -> str:
    return lib().px_last_error().decode()


def version() -> str:
    return lib().px_version().decode()


def dtype_code(t: torch.Tensor) -> int:
    try:
        return _DTYPE_CODE[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype} (float64, float32, bfloat16)")


def _stream_handle(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ld(t: torch.Tensor, rows: int, min_cols: int, name: str) -> int:
    if t.dim() != 2 or t.shape[0] != rows or t.shape[1] < min_cols or t.stride(1) != 1:
        raise ValueError(f"{name}: expected a ({rows}, >={min_cols}) tensor with unit column stride, "
                         f"got shape {tuple(t.shape)} strides {t.stride()}")
    ld = t.stride(0)
    need = (t.storage_offset() + rows * ld) * t.element_size()
    if t.untyped_storage().nbytes() < need:
        raise ValueError(f"{name}: storage holds fewer than rows*ld elements")
    return ld


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


# ------------------------------------------------------------------ memory --

def round_up(x: int, m: int) -> int:
    return (x + m - 1) // m * m


def alloc_grid(n: int, dtype=torch.float64, device="cuda", ld: int | None = None) -> torch.Tensor:
    """Zeroed (n+2) x ld grid; default ld = n+2 rounded up to 128 bytes."""
    es = torch.empty(0, dtype=dtype).element_size()
    ld = ld or round_up(n + 2, 128 // es)
    return torch.zeros((n + 2, ld), dtype=dtype, device=device)


def alloc_rhs(n: int, dtype=torch.float64, device="cuda", ld_f: int | None = None) -> torch.Tensor:
    """Zeroed n x ld_f right-hand side; default ld_f = n rounded up to 128 bytes (rows
    16-byte aligned, so the relaxation kernels use vector loads)."""
    es = torch.empty(0, dtype=dtype).element_size()
    ld_f = ld_f or round_up(n, 128 // es)
    return torch.zeros((n, ld_f), dtype=dtype, device=device)


# ----------------------------------------------------------------- context --

class Context:
    """Owns a px_ctx (scratch memory for relaxation and reductions)."""

    def __init__(self, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        h = ctypes.c_void_p()
        _check(lib().px_ctx_create(int(device), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def reserve(self, n: int, ld: int, dtype: int):
        _check(lib().px_ctx_reserve(self._h, n, ld, dtype))

    def set_tile_rows(self, rows: int):
        _check(lib().px_ctx_set_tile_rows(self._h, int(rows)))

    def close(self):
        if self._h:
            lib().px_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------- operations --

def apply_stencil(phi, n, out, taps=LAPLACE_TAPS, scale=1.0, bc=BC_DIRICHLET0, stream=None):
    """out = scale * S(phi) over the interior (Eq. 1, 3x3 taps)."""
    ld = _ld(phi, n + 2, n + 2, "phi")
    ldo = _ld(out, n, n, "out")
    if out.dtype != phi.dtype:
        raise TypeError("out must have phi's dtype")
    t = (ctypes.c_double * 9)(*[float(x) for x in taps])
    _check(lib().px_apply_stencil(_ptr(phi), n, ld, dtype_code(phi), _ptr(out), ldo, t, float(scale),
                                  int(bc), _stream_handle(stream)))
    return out


def residual(phi, n, f, h, norms, ctx: Context, bc=BC_DIRICHLET0, r=None, stream=None):
    """r = f - (1/h^2) S(phi); norms (float64 device tensor of 2) <- {max|r|, sum r^2}."""
    ld = _ld(phi, n + 2, n + 2, "phi")
    ldf = _ld(f, n, n, "f")
    ldr = _ld(r, n, n, "r") if r is not None else 0
    _check(lib().px_residual(_ptr(phi), n, ld, dtype_code(phi), _ptr(f), ldf, float(h), int(bc),
                             _ptr(r), ldr, _ptr(norms), ctx.handle, _stream_handle(stream)))
    return norms


def jacobi_update(phi, n, s, f, h, lam, stream=None):
    """In place: phi = (phi + (lam/h^2) s) - lam f over the interior (unfused step)."""
    ld = _ld(phi, n + 2, n + 2, "phi")
    lds = _ld(s, n, n, "s")
    ldf = _ld(f, n, n, "f")
    _check(lib().px_jacobi_update(_ptr(phi), n, ld, dtype_code(phi), _ptr(s), lds, _ptr(f), ldf,
                                  float(h), float(lam), _stream_handle(stream)))
    return phi


def relax_fused(phi_in, phi_out, n, f, h, lam, nsweeps, ctx: Context, tblock=0,
                bc=BC_DIRICHLET0, resmode=RES_FINAL, norms=None, stream=None):
    """nsweeps fused damped-Jacobi sweeps phi_in -> phi_out (tblock sweeps per launch)."""
    ld = _ld(phi_in, n + 2, n + 2, "phi_in")
    if _ld(phi_out, n + 2, n + 2, "phi_out") != ld:
        raise ValueError("phi_in and phi_out must share ld")
    ldf = _ld(f, n, n, "f")
    _check(lib().px_relax_fused(_ptr(phi_in), _ptr(phi_out), n, ld, dtype_code(phi_in), _ptr(f), ldf,
                                float(h), float(lam), int(nsweeps), int(tblock), int(bc), int(resmode),
                                _ptr(norms), ctx.handle, _stream_handle(stream)))
    return phi_out


def relax_fused_noalloc(phi_in, phi_out, n, f, h, lam, nsweeps, bc=BC_DIRICHLET0, resmode=RES_FINAL,
                       norms=None, stream=None):
    """One launch of 1..8 fused sweeps phi_in -> phi_out with no context: the library
    allocates nothing (its reduction partials sit in a fixed device array)."""
    ld = _ld(phi_in, n + 2, n + 2, "phi_in")
    if _ld(phi_out, n + 2, n + 2, "phi_out") != ld:
        raise ValueError("phi_in and phi_out must share ld")
    ldf = _ld(f, n, n, "f")
    _check(lib().px_relax_fused_noalloc(_ptr(phi_in), _ptr(phi_out), n, ld, dtype_code(phi_in), _ptr(f), ldf,
                                        float(h), float(lam), int(nsweeps), int(bc), int(resmode), _ptr(norms),
                                        _stream_handle(stream)))
    return phi_out


def autotune(phi_in, phi_out, n, f, ctx: Context, bc=BC_DIRICHLET0, stream=None):
    """Times (sweeps per launch, tile rows) candidates on these buffers and stores the
    fastest in ctx for this grid; returns (k, rows, Gcell-updates/s of the winner)."""
    ld = _ld(phi_in, n + 2, n + 2, "phi_in")
    if _ld(phi_out, n + 2, n + 2, "phi_out") != ld:
        raise ValueError("phi_in and phi_out must share ld")
    ldf = _ld(f, n, n, "f")
    k, rows, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(lib().px_autotune(_ptr(phi_in), _ptr(phi_out), n, ld, dtype_code(phi_in), _ptr(f), ldf,
                             int(bc), ctx.handle, _stream_handle(stream), ctypes.byref(k),
                             ctypes.byref(rows), ctypes.byref(g)))
    return k.value, rows.value, g.value


@dataclass
class SolveStats:
    status: int
    sweeps: int
    outer_steps: int
    res_max: float
    res_l2: float
    rel_res_max: float
    rel_res_l2: float
    seconds: float


def solve(phi, n, f, h, lam, ctx: Context, mode=SOLVE_PLAIN, rtol=1e-10, norm=0,
          max_sweeps=10 ** 9, check_every=0, inner_sweeps=0, tblock=0, bc=BC_DIRICHLET0,
          stream=None, raise_on_error=True) -> SolveStats:
    """Iterate to ||r|| <= rtol ||f|| in place on phi; returns the solve statistics."""
    ld = _ld(phi, n + 2, n + 2, "phi")
    ldf = _ld(f, n, n, "f")
    o = _SolveOpts(int(mode), int(norm), float(rtol), int(max_sweeps), int(check_every),
                   int(inner_sweeps), int(tblock), int(bc))
    s = _SolveStats()
    st = lib().px_solve(_ptr(phi), n, ld, dtype_code(phi), _ptr(f), ldf, float(h), float(lam),
                        ctypes.byref(o), ctypes.byref(s), ctx.handle, _stream_handle(stream))
    if st != OK and raise_on_error:
        _check(st)
    return SolveStats(st, s.sweeps, s.outer_steps, s.res_max, s.res_l2, s.rel_res_max, s.rel_res_l2,
                      s.seconds)


# ----------------------------------------------------------------- batches --

def _problems(items):
    """items: sequence of (phi, f, n, h, lam); returns a ctypes array of px_problem."""
    arr = (_Problem * len(items))()
    dt = None
    for k, (phi, f, n, h, lam) in enumerate(items):
        ld = _ld(phi, n + 2, n + 2, f"phi[{k}]")
        ldf = _ld(f, n, n, f"f[{k}]")
        if dt is None:
            dt = phi.dtype
        if phi.dtype != dt or f.dtype != dt:
            raise TypeError("every phi and f of a batch must share one dtype")
        arr[k] = _Problem(phi.data_ptr(), f.data_ptr(), n, ld, ldf, float(h), float(lam))
    return arr, dt


def relax_batched(items, nsweeps, ctx: Context, tblock=0, bc=BC_DIRICHLET0, resmode=RES_FINAL,
                  norms=None, stream=None):
    """nsweeps fused sweeps on every (phi, f, n, h, lam) of the batch, in place; norms
    (float64 device tensor of 2*len(items)) gets each problem's final {max|r|, sum r^2}."""
    arr, dt = _problems(items)
    _check(lib().px_relax_batched(arr, len(items), _DTYPE_CODE[dt], int(nsweeps), int(tblock), int(bc),
                                  int(resmode), _ptr(norms), ctx.handle, _stream_handle(stream)))


def relax_boxes(items, nbx, nby, nsweeps, ctx: Context, exchange=1, bc=BC_DIRICHLET0, stream=None):
    """One domain of nbx x nby boxes (items in box-row-major order, each (phi, f, n, h, lam)
    with the same n, h and lam): ghost rings refreshed from the neighbouring boxes every
    `exchange` sweeps, then each box relaxed with fixed ghosts; in place."""
    arr, dt = _problems(items)
    _check(lib().px_relax_boxes(arr, int(nbx), int(nby), _DTYPE_CODE[dt], int(nsweeps), int(exchange), int(bc), ctx.handle,
                                _stream_handle(stream)))


def autotune_batched(items, ctx: Context, bc=BC_DIRICHLET0, stream=None) -> int:
    """Tunes tile rows per problem size and sweeps per launch for batches of these
    problems' dtype (relaxes them in place while timing); returns the chosen k."""
    arr, dt = _problems(items)
    k = ctypes.c_int()
    _check(lib().px_autotune_batched(arr, len(items), _DTYPE_CODE[dt], int(bc), ctx.handle,
                                     _stream_handle(stream), ctypes.byref(k)))
    return k.value


def solve_batched(items, ctx: Context, mode=SOLVE_MIXED_F32, rtol=1e-8, norm=0, max_sweeps=10 ** 9,
                  inner_sweeps=0, tblock=0, bc=BC_DIRICHLET0, stream=None, raise_on_error=True):
    """FP64-refined mixed-precision solve of every (phi, f, n, h, lam) (float64) in place;
    returns (status, [SolveStats per problem])."""
    arr, _ = _problems(items)
    o = _SolveOpts(int(mode), int(norm), float(rtol), int(max_sweeps), 0, int(inner_sweeps),
                   int(tblock), int(bc))
    st = (_SolveStats * len(items))()
    status = lib().px_solve_batched(arr, len(items), ctypes.byref(o), st, ctx.handle,
                                    _stream_handle(stream))
    if status != OK and raise_on_error:
        _check(status)
    return status, [SolveStats(status, x.sweeps, x.outer_steps, x.res_max, x.res_l2, x.rel_res_max,
                               x.rel_res_l2, x.seconds) for x in st]


# ---------------------------------------------------- learned correction --

NET_NPARAM = 19008
LOSS_MSE, LOSS_ENERGY = 0, 1


def _host_f32(w):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(w, dtype=np.float32).ravel())
    if a.size != NET_NPARAM:
        raise ValueError(f"expected {NET_NPARAM} weights, got {a.size}")
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Net:
    """Owns a px_net: the 4-layer 3x3 correction network, its FP32 master weights,
    BF16 copies, Adam state and activation workspace on one device."""

    def __init__(self, weights, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        a, p = _host_f32(weights)
        h = ctypes.c_void_p()
        _check(lib().px_net_create(int(device), p, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def set_weights(self, weights):
        a, p = _host_f32(weights)
        _check(lib().px_net_set_weights(self._h, p))

    def get_weights(self):
        import numpy as np
        a = np.zeros(NET_NPARAM, dtype=np.float32)
        _check(lib().px_net_get_weights(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return a

    def forward(self, x, y, x_scale=1.0, stream=None, infer=False):
        """y = N(x * x_scale); x: (B, H, ldx) or (H, ldx) float64/float32 with unit column
        stride (the first W columns used, W = y's width); y: float32 of shape (B, H, >= W).
        infer=True: the same y through px_net_infer (layers 1 and 2 fused, hidden
        activations not kept)."""
        x3 = x if x.dim() == 3 else x.unsqueeze(0)
        y3 = y if y.dim() == 3 else y.unsqueeze(0)
        B, H, W = y3.shape[0], y3.shape[1], y3.shape[2]
        if x3.dtype not in (torch.float64, torch.float32) or y3.dtype != torch.float32:
            raise TypeError("x must be float64 or float32 and y float32")
        if x3.shape[0] != B or x3.shape[1] != H or x3.stride(2) != 1 or y3.stride(2) != 1:
            raise ValueError("x and y must have matching batch and rows, unit column stride")
        ldx, ldy = x3.stride(1), y3.stride(1)
        if x3.stride(0) != H * ldx or y3.stride(0) != H * ldy:
            raise ValueError("images must be stored back to back (stride(0) == H * stride(1))")
        fn = lib().px_net_infer if infer else lib().px_net_forward
        _check(fn(self._h, _ptr(x3), dtype_code(x3), ldx, B, H, W, float(x_scale), _ptr(y3), ldy,
                  _stream_handle(stream)))
        return y

    def loss_grad(self, x, t, loss=LOSS_MSE, loss_out=None, grad=None, stream=None):
        """Forward, loss and backward on contiguous float32 (B, H, W) x and targets t; the
        gradient stays in the network (and is copied to grad if given)."""
        if x.dtype != torch.float32 or t.dtype != torch.float32 or not x.is_contiguous() \
                or not t.is_contiguous() or x.shape != t.shape or x.dim() != 3:
            raise ValueError("x and t must be contiguous float32 tensors of one (B, H, W) shape")
        B, H, W = x.shape
        _check(lib().px_net_loss_grad(self._h, _ptr(x), _ptr(t), B, H, W, int(loss), _ptr(loss_out),
                                      _ptr(grad), _stream_handle(stream)))

    def adam(self, lr, stream=None):
        _check(lib().px_net_adam(self._h, ctypes.c_float(lr), _stream_handle(stream)))

    def activation(self, layer, out, stream=None):
        """Copy layer 1..3 of the last forward pass (bfloat16 bits as int16/uint16, shape
        (pixels, 32)) into out."""
        _check(lib().px_net_activation(self._h, int(layer), _ptr(out), _stream_handle(stream)))
        return out

    def close(self):
        if self._h:
            lib().px_net_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_pair(phi, n, x, t, ctx: Context, loss=LOSS_MSE, stream=None):
    """Training pair of the homogeneous problem: x = r / rms(r), t = e / rms(e) (or the
    energy-norm scaling) with e = -phi, r = -L phi; x and t contiguous float32 (n, n)."""
    ld = _ld(phi, n + 2, n + 2, "phi")
    if phi.dtype != torch.float64:
        raise TypeError("phi must be float64")
    for a, nm in ((x, "x"), (t, "t")):
        if a.dtype != torch.float32 or not a.is_contiguous() or a.numel() != n * n:
            raise ValueError(f"{nm} must be a contiguous float32 tensor of n*n elements")
    _check(lib().px_net_make_pair(_ptr(phi), n, ld, int(loss), _ptr(x), _ptr(t), ctx.handle,
                                  _stream_handle(stream)))


def correction_step(phi, n, r, d, h, ctx: Context, mode=2, coef=None, stream=None):
    """phi += a r + b d with the energy-optimal (a, b) for mode (0: r, 1: d, 2: both);
    r float64 (n, >= n), d float64/float32 (n, >= n) or None (mode 0); coef: float64
    device tensor of 2 receiving (a, b), or None."""
    ld = _ld(phi, n + 2, n + 2, "phi")
    ldr = _ld(r, n, n, "r")
    if d is None:
        dp, ddt, ldd = ctypes.c_void_p(0), F64, 0
    else:
        dp, ddt, ldd = _ptr(d), dtype_code(d), _ld(d, n, n, "d")
    _check(lib().px_correction_step(_ptr(phi), n, ld, _ptr(r), ldr, dp, ddt, ldd, float(h), int(mode),
                                    _ptr(coef), ctx.handle, _stream_handle(stream)))


@dataclass
class LearnedStats(SolveStats):
    corrections: int = 0
    rejected: int = 0
    fell_back: int = 0
    discarded_sweeps: int = 0  # sweeps of undone steps (included in sweeps)


def solve_learned(phi, n, f, h, lam, ctx: Context, net: "Net | None" = None, use_net=1, rtol=1e-10,
                  norm=0, max_sweeps=10 ** 9, smooth_sweeps=16, tblock=0, judge=2, stream=None,
                  raise_on_error=True) -> LearnedStats:
    """Refinement loop with energy-optimal correction steps along r (use_net 0), the
    network's direction (1) or both (2), plain smoothing sweeps and the plain-relaxation
    judge; float64 phi and f, in place."""
    ld = _ld(phi, n + 2, n + 2, "phi")
    ldf = _ld(f, n, n, "f")
    o = _LearnedOpts(int(norm), float(rtol), int(max_sweeps), int(smooth_sweeps), int(tblock), int(use_net),
                     int(judge))
    s = _LearnedStats()
    st = lib().px_solve_learned(_ptr(phi), n, ld, _ptr(f), ldf, float(h), float(lam),
                                net.handle if net is not None else ctypes.c_void_p(0), ctypes.byref(o),
                                ctypes.byref(s), ctx.handle, _stream_handle(stream))
    if st != OK and raise_on_error:
        _check(st)
    b = s.base
    return LearnedStats(st, b.sweeps, b.outer_steps, b.res_max, b.res_l2, b.rel_res_max, b.rel_res_l2,
                        b.seconds, s.corrections, s.rejected, s.fell_back, s.discarded_sweeps)
