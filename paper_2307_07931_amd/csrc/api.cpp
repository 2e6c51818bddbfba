// api.cpp -- the C ABI declared in include/protox.h: argument validation (on
// the host, before any HIP call), the context and its scratch memory, launch
// sequencing for multi-launch relaxation, and the host-driven solve loop.
#include "../../include/protox.h"
#include "px_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

using namespace px;

struct px_tuned {
    int n = 0, ld = 0, k = 0, rows = 0;
    int rows_norm = 0;  // tile rows for the launches of k sweeps that also take the norms
    double gcells = 0.0;
};

struct px_ctx {
    int device = 0;
    int tile_rows = 0;
    px_tuned tuned[3];  // per dtype: autotuned (k, rows) for one (n, ld)
    // ping-pong grid (any dtype) for multi-launch relaxation
    void *grid = nullptr;
    size_t grid_bytes = 0;
    // reduction partials: count slots of (u64 max bits, double sum)
    unsigned long long *pmax = nullptr;
    double *psum = nullptr;
    size_t part_count = 0;
    // solve: device norms, pinned host copy, norms of f
    double *norms_dev = nullptr;
    double *norms_host = nullptr;
    // mixed precision: FP64 second grid, two low-precision ghosted grids, low r
    void *mix = nullptr;
    size_t mix_bytes = 0;
    // batched calls
    BatchWork *batch = nullptr;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(PX_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define PX_HIP(call, what)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return hip_fail(e_, what);                                          \
    } while (0)

constexpr int MAX_N = 1 << 17;

bool valid_dtype(int d) { return d == F64 || d == F32 || d == BF16; }
bool valid_bc(int b) { return b == DIRICHLET0 || b == GHOST_FIXED || b == PERIODIC; }

size_t grid_bytes(int n, int ld, int dtype) { return (size_t)(n + 2) * (size_t)ld * elem_size(dtype); }
size_t flat_bytes(int n, int ld, int dtype) { return (size_t)n * (size_t)ld * elem_size(dtype); }

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

int check_n_ld(int n, int ld, int dtype)
{
    if (!valid_dtype(dtype)) return fail(PX_EINVAL, "unknown dtype %d", dtype);
    if (n < 1 || n > MAX_N) return fail(PX_EINVAL, "n = %d outside [1, %d]", n, MAX_N);
    if (ld < n + 2) return fail(PX_EINVAL, "ld = %d < n + 2 = %d", ld, n + 2);
    return PX_OK;
}

int check_ptr(const void *p, int dtype, const char *name)
{
    if (!p) return fail(PX_EINVAL, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) % (uintptr_t)elem_size(dtype))
        return fail(PX_EINVAL, "%s is not aligned to its element size", name);
    return PX_OK;
}

int check_flat(const void *p, int n, int ldx, int dtype, const char *name)
{
    int st = check_ptr(p, dtype, name);
    if (st) return st;
    if (ldx < n) return fail(PX_EINVAL, "leading dimension of %s (%d) < n (%d)", name, ldx, n);
    return PX_OK;
}

int check_pos(double x, const char *name)
{
    if (!(x > 0.0) || !std::isfinite(x)) return fail(PX_EINVAL, "%s must be positive and finite", name);
    return PX_OK;
}

int set_device(px_ctx *ctx)
{
    PX_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    return PX_OK;
}

int ensure_grid(px_ctx *ctx, size_t bytes)
{
    if (ctx->grid_bytes >= bytes) return PX_OK;
    if (ctx->grid) (void)hipFree(ctx->grid);
    ctx->grid = nullptr;
    ctx->grid_bytes = 0;
    if (hipMalloc(&ctx->grid, bytes) != hipSuccess) return fail(PX_ENOMEM, "hipMalloc(%zu) failed", bytes);
    ctx->grid_bytes = bytes;
    return PX_OK;
}

int ensure_partials(px_ctx *ctx, size_t count)
{
    if (ctx->part_count >= count) return PX_OK;
    if (ctx->pmax) (void)hipFree(ctx->pmax);
    if (ctx->psum) (void)hipFree(ctx->psum);
    ctx->pmax = nullptr;
    ctx->psum = nullptr;
    ctx->part_count = 0;
    if (hipMalloc(&ctx->pmax, count * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&ctx->psum, count * sizeof(double)) != hipSuccess)
        return fail(PX_ENOMEM, "hipMalloc of %zu reduction partials failed", count);
    ctx->part_count = count;
    return PX_OK;
}

int ensure_norms(px_ctx *ctx)
{
    if (ctx->norms_dev) return PX_OK;
    if (hipMalloc(&ctx->norms_dev, 8 * sizeof(double)) != hipSuccess)
        return fail(PX_ENOMEM, "hipMalloc(norms) failed");
    if (hipHostMalloc(&ctx->norms_host, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess)
        return fail(PX_ENOMEM, "hipHostMalloc(norms) failed");
    return PX_OK;
}

int ensure_mix(px_ctx *ctx, size_t bytes)
{
    if (ctx->mix_bytes >= bytes) return PX_OK;
    if (ctx->mix) (void)hipFree(ctx->mix);
    ctx->mix = nullptr;
    ctx->mix_bytes = 0;
    if (hipMalloc(&ctx->mix, bytes) != hipSuccess) return fail(PX_ENOMEM, "hipMalloc(%zu) failed", bytes);
    ctx->mix_bytes = bytes;
    return PX_OK;
}

const px_tuned *tuned_for(const px_ctx *ctx, int dtype, int n, int ld)
{
    const px_tuned &t = ctx->tuned[dtype];
    return (t.k > 0 && t.n == n && t.ld == ld) ? &t : nullptr;
}

int default_tblock(const px_ctx *ctx, int dtype, int n, int ld)
{
    if (const px_tuned *t = tuned_for(ctx, dtype, n, ld)) return t->k;
    // untuned: 8 sweeps per launch was fastest at every size measured (large grids:
    // fewest passes over HBM; small grids: fewest launches)
    return 8;
}

// Tile height for a launch of `ks` sweeps (residual mode rm): explicit override, then the
// tuned value (when the tuned k is the one launched; launches with norms have their own),
// then the built-in default.
int pick_rows(const px_ctx *ctx, int dtype, int n, int ld, int ks, int rm = RES_NONE)
{
    if (ctx->tile_rows > 0) return ctx->tile_rows;
    if (const px_tuned *t = tuned_for(ctx, dtype, n, ld))
        if (t->k == ks) return (rm != RES_NONE && t->rows_norm > 0) ? t->rows_norm : t->rows;
    return relax_default_rows(dtype, n, ks);
}

Partials partials(px_ctx *ctx) { return Partials{ctx->pmax, ctx->psum}; }

// Runs nsweeps sweeps: src -> ... -> dst, alternating between dst and tmp so the
// last launch writes dst.  src is only read.  tmp may be NULL when one launch.
int run_sweeps(px_ctx *ctx, int dtype, const void *src, void *dst, void *tmp, int n, int ld,
               const void *f, int ld_f, double h, double lambda, int nsweeps, int k, int bc,
               int resmode, double *norms, hipStream_t s, int forced_rows = 0, int forced_rows_norm = 0)
{
    const int L = (nsweeps + k - 1) / k;
    const double c = 1.0 / (h * h);
    const double w = lambda / (h * h);
    const void *cur = src;
    int done = 0;
    for (int i = 0; i < L; ++i) {
        const int ks = std::min(k, nsweeps - done);
        void *to = (((L - 1 - i) % 2) == 0) ? dst : tmp;
        RelaxLaunch a;
        a.in = cur;
        a.out = to;
        a.f = f;
        a.n = n;
        a.ld = ld;
        a.ld_f = ld_f;
        a.c = c;
        a.w = w;
        a.lam = lambda;
        a.bc = bc;
        a.sweeps = ks;
        a.resmode = (i == L - 1) ? resmode : RES_NONE;
        const int forced = (a.resmode != RES_NONE && forced_rows_norm > 0) ? forced_rows_norm : forced_rows;
        a.rows = forced > 0 ? forced : pick_rows(ctx, dtype, n, ld, ks, a.resmode);
        a.part = partials(ctx);
        if (a.resmode != RES_NONE) {
            int st = ensure_partials(ctx, (size_t)relax_num_waves(dtype, n, ks, a.resmode, a.rows));
            if (st) return st;
            a.part = partials(ctx);
        }
        PX_HIP(relax_launch(dtype, a, s), "relax kernel launch");
        if (a.resmode != RES_NONE)
            PX_HIP(reduce_partials(a.part, relax_num_waves(dtype, n, ks, a.resmode, a.rows), norms, s),
                   "norm reduction launch");
        cur = to;
        done += ks;
    }
    return PX_OK;
}

int residual_into(px_ctx *ctx, int dtype, const void *phi, int n, int ld, const void *f, int ld_f,
                  double h, int bc, void *r, int ld_r, double *norms, hipStream_t s)
{
    const int nblk = pointwise_num_blocks(n);
    int st = ensure_partials(ctx, (size_t)nblk);
    if (st) return st;
    PX_HIP(residual_launch(dtype, phi, n, ld, f, ld_f, 1.0 / (h * h), bc, r, ld_r, partials(ctx), s),
           "residual kernel launch");
    PX_HIP(reduce_partials(partials(ctx), nblk, norms, s), "norm reduction launch");
    return PX_OK;
}

}  // namespace

int px::set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

extern "C" {

const char *px_last_error(void) { return g_err.c_str(); }
const char *px_version(void) { return "protox-mi355x 0.1 (gfx950)"; }

int px_ctx_create(int device, px_ctx **out)
{
    if (!out) return fail(PX_EINVAL, "out is NULL");
    if (device < 0) return fail(PX_EINVAL, "device %d < 0", device);
    px_ctx *c = new (std::nothrow) px_ctx();
    if (!c) return fail(PX_ENOMEM, "out of host memory");
    c->device = device;
    *out = c;
    return PX_OK;
}

int px_ctx_destroy(px_ctx *ctx)
{
    if (!ctx) return PX_OK;
    if (ctx->grid || ctx->pmax || ctx->norms_dev || ctx->mix) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        if (ctx->grid) (void)hipFree(ctx->grid);
        if (ctx->pmax) (void)hipFree(ctx->pmax);
        if (ctx->psum) (void)hipFree(ctx->psum);
        if (ctx->norms_dev) (void)hipFree(ctx->norms_dev);
        if (ctx->norms_host) (void)hipHostFree(ctx->norms_host);
        if (ctx->mix) (void)hipFree(ctx->mix);
    }
    if (ctx->batch) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        delete ctx->batch;
    }
    delete ctx;
    return PX_OK;
}

int px_ctx_set_tile_rows(px_ctx *ctx, int rows)
{
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    if (rows < 0 || rows > 4096) return fail(PX_EINVAL, "tile rows %d outside [0, 4096]", rows);
    ctx->tile_rows = rows;
    return PX_OK;
}

int px_ctx_reserve(px_ctx *ctx, int n, int ld, int dtype)
{
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    int st = check_n_ld(n, ld, dtype);
    if (st) return st;
    if ((st = set_device(ctx))) return st;
    if ((st = ensure_grid(ctx, grid_bytes(n, ld, dtype)))) return st;
    size_t parts = (size_t)pointwise_num_blocks(n);
    for (int k = 1; k <= 8; ++k)
        for (int rm = RES_LAGGED; rm <= RES_FINAL; ++rm) {
            parts = std::max(parts, (size_t)relax_num_waves(dtype, n, k, rm, pick_rows(ctx, dtype, n, ld, k, rm)));
        }
    if ((st = ensure_partials(ctx, parts))) return st;
    return ensure_norms(ctx);
}

int px_apply_stencil(const void *phi, int n, int ld, int dtype, void *out, int ld_out,
                     const double *taps, double scale, int bc, void *stream)
{
    int st = check_n_ld(n, ld, dtype);
    if (st) return st;
    if ((st = check_ptr(phi, dtype, "phi"))) return st;
    if ((st = check_flat(out, n, ld_out, dtype, "out"))) return st;
    if (!taps) return fail(PX_EINVAL, "taps is NULL");
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(taps[k])) return fail(PX_EINVAL, "tap %d is not finite", k);
    if (!std::isfinite(scale)) return fail(PX_EINVAL, "scale is not finite");
    if (!valid_bc(bc)) return fail(PX_EINVAL, "unknown bc %d", bc);
    if (overlap(phi, grid_bytes(n, ld, dtype), out, flat_bytes(n, ld_out, dtype)))
        return fail(PX_EALIAS, "out overlaps phi");
    PX_HIP(stencil_launch(dtype, phi, n, ld, out, ld_out, taps, scale, bc, (hipStream_t)stream),
           "stencil kernel launch");
    return PX_OK;
}

int px_residual(const void *phi, int n, int ld, int dtype, const void *f, int ld_f, double h,
                int bc, void *r, int ld_r, double *norms, px_ctx *ctx, void *stream)
{
    int st = check_n_ld(n, ld, dtype);
    if (st) return st;
    if ((st = check_ptr(phi, dtype, "phi"))) return st;
    if ((st = check_flat(f, n, ld_f, dtype, "f"))) return st;
    if (r && (st = check_flat(r, n, ld_r, dtype, "r"))) return st;
    if (!norms) return fail(PX_EINVAL, "norms is NULL");
    if (reinterpret_cast<uintptr_t>(norms) % 8) return fail(PX_EINVAL, "norms is not 8-byte aligned");
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    if ((st = check_pos(h, "h"))) return st;
    if (!valid_bc(bc)) return fail(PX_EINVAL, "unknown bc %d", bc);
    if (r && (overlap(r, flat_bytes(n, ld_r, dtype), phi, grid_bytes(n, ld, dtype)) ||
              overlap(r, flat_bytes(n, ld_r, dtype), f, flat_bytes(n, ld_f, dtype))))
        return fail(PX_EALIAS, "r overlaps phi or f");
    if ((st = set_device(ctx))) return st;
    return residual_into(ctx, dtype, phi, n, ld, f, ld_f, h, bc, r, ld_r, norms, (hipStream_t)stream);
}

int px_jacobi_update(void *phi, int n, int ld, int dtype, const void *s, int ld_s, const void *f,
                     int ld_f, double h, double lambda, void *stream)
{
    int st = check_n_ld(n, ld, dtype);
    if (st) return st;
    if ((st = check_ptr(phi, dtype, "phi"))) return st;
    if ((st = check_flat(s, n, ld_s, dtype, "s"))) return st;
    if ((st = check_flat(f, n, ld_f, dtype, "f"))) return st;
    if ((st = check_pos(h, "h")) || (st = check_pos(lambda, "lambda"))) return st;
    if (overlap(phi, grid_bytes(n, ld, dtype), s, flat_bytes(n, ld_s, dtype)) ||
        overlap(phi, grid_bytes(n, ld, dtype), f, flat_bytes(n, ld_f, dtype)))
        return fail(PX_EALIAS, "phi overlaps s or f");
    PX_HIP(jacobi_launch(dtype, phi, n, ld, s, ld_s, f, ld_f, lambda / (h * h), lambda,
                         (hipStream_t)stream),
           "jacobi kernel launch");
    return PX_OK;
}

int px_relax_fused(const void *phi_in, void *phi_out, int n, int ld, int dtype, const void *f,
                   int ld_f, double h, double lambda, int nsweeps, int tblock, int bc, int resmode,
                   double *norms, px_ctx *ctx, void *stream)
{
    int st = check_n_ld(n, ld, dtype);
    if (st) return st;
    if ((st = check_ptr(phi_in, dtype, "phi_in")) || (st = check_ptr(phi_out, dtype, "phi_out")))
        return st;
    if ((st = check_flat(f, n, ld_f, dtype, "f"))) return st;
    if ((st = check_pos(h, "h")) || (st = check_pos(lambda, "lambda"))) return st;
    if (nsweeps < 0) return fail(PX_EINVAL, "nsweeps = %d < 0", nsweeps);
    if (tblock < 0 || tblock > 8) return fail(PX_EINVAL, "tblock = %d outside [0, 8]", tblock);
    if (!valid_bc(bc)) return fail(PX_EINVAL, "unknown bc %d", bc);
    if (resmode < RES_NONE || resmode > RES_FINAL) return fail(PX_EINVAL, "unknown resmode %d", resmode);
    if (resmode != RES_NONE && !norms) return fail(PX_EINVAL, "norms is NULL");
    if (norms && reinterpret_cast<uintptr_t>(norms) % 8) return fail(PX_EINVAL, "norms is not 8-byte aligned");
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    const size_t gb = grid_bytes(n, ld, dtype);
    if (overlap(phi_in, gb, phi_out, gb)) return fail(PX_EALIAS, "phi_out overlaps phi_in");
    if (overlap(f, flat_bytes(n, ld_f, dtype), phi_out, gb)) return fail(PX_EALIAS, "phi_out overlaps f");
    if ((st = set_device(ctx))) return st;
    hipStream_t s = (hipStream_t)stream;
    if (nsweeps == 0) {
        PX_HIP(copy_grid_launch(dtype, phi_in, phi_out, n, ld, s), "copy kernel launch");
        if (resmode != RES_NONE)
            return residual_into(ctx, dtype, phi_in, n, ld, f, ld_f, h, bc, nullptr, 0, norms, s);
        return PX_OK;
    }
    const int k = tblock ? tblock : default_tblock(ctx, dtype, n, ld);
    void *tmp = nullptr;
    if ((nsweeps + k - 1) / k > 1) {
        if ((st = ensure_grid(ctx, gb))) return st;
        tmp = ctx->grid;
    }
    return run_sweeps(ctx, dtype, phi_in, phi_out, tmp, n, ld, f, ld_f, h, lambda, nsweeps, k, bc,
                      resmode, norms, s);
}

}  // extern "C"

// ---- relaxation without allocation ---------------------------------------------------
// Reduction partials of px_relax_fused_noalloc: a fixed device array, one copy per GPU the
// library runs on, held until the process ends.  Slots [0, NOALLOC_PARTIALS) hold the
// max|r| bit patterns, [NOALLOC_PARTIALS, 2 NOALLOC_PARTIALS) the sums of squares.  Every
// tile of a launch writes its own slot before the reduction reads it, so nothing needs
// clearing between calls.  The array's name is only a host-side handle: kernels get the
// address hipGetSymbolAddress returns for the current device.
constexpr int NOALLOC_PARTIALS = PX_NOALLOC_MAX_PARTIALS;
static __device__ __align__(256) unsigned long long scratch[2 * NOALLOC_PARTIALS];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[NOALLOC_MAX_DEVICES];

// The device address of `scratch` on the current device (looked up once per device).
int noalloc_scratch(void **out)
{
    int dev = -1;
    PX_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(PX_EUNSUPPORTED, "device %d beyond the %d devices the library supports", dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        PX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(PX_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return PX_OK;
}

}  // namespace

extern "C" {

int px_relax_fused_noalloc(const void *phi_in, void *phi_out, int n, int ld, int dtype, const void *f,
                           int ld_f, double h, double lambda, int nsweeps, int bc, int resmode, double *norms,
                           void *stream)
{
    int st = check_n_ld(n, ld, dtype);
    if (st) return st;
    if ((st = check_ptr(phi_in, dtype, "phi_in")) || (st = check_ptr(phi_out, dtype, "phi_out")))
        return st;
    if ((st = check_flat(f, n, ld_f, dtype, "f"))) return st;
    if ((st = check_pos(h, "h")) || (st = check_pos(lambda, "lambda"))) return st;
    if (nsweeps < 1 || nsweeps > 8)
        return fail(PX_EINVAL, "nsweeps = %d outside [1, 8] (one launch; no ping-pong buffer)", nsweeps);
    if (!valid_bc(bc)) return fail(PX_EINVAL, "unknown bc %d", bc);
    if (resmode < RES_NONE || resmode > RES_FINAL) return fail(PX_EINVAL, "unknown resmode %d", resmode);
    if (resmode != RES_NONE && !norms) return fail(PX_EINVAL, "norms is NULL");
    if (norms && reinterpret_cast<uintptr_t>(norms) % 8) return fail(PX_EINVAL, "norms is not 8-byte aligned");
    const size_t gb = grid_bytes(n, ld, dtype);
    if (overlap(phi_in, gb, phi_out, gb)) return fail(PX_EALIAS, "phi_out overlaps phi_in");
    if (overlap(f, flat_bytes(n, ld_f, dtype), phi_out, gb)) return fail(PX_EALIAS, "phi_out overlaps f");
    const int rows = relax_default_rows(dtype, n, nsweeps);
    const int parts = relax_num_waves(dtype, n, nsweeps, resmode, rows);
    if (resmode != RES_NONE && parts > NOALLOC_PARTIALS)
        return fail(PX_EINVAL, "grid of n = %d needs %d reduction partials; the fixed scratch holds %d", n, parts,
                    NOALLOC_PARTIALS);
    void *base = nullptr;
    if ((st = noalloc_scratch(&base))) return st;
    RelaxLaunch a;
    a.in = phi_in;
    a.out = phi_out;
    a.f = f;
    a.n = n;
    a.ld = ld;
    a.ld_f = ld_f;
    a.c = 1.0 / (h * h);
    a.w = lambda / (h * h);
    a.lam = lambda;
    a.bc = bc;
    a.sweeps = nsweeps;
    a.resmode = resmode;
    a.rows = rows;
    a.part = Partials{static_cast<unsigned long long *>(base),
                      reinterpret_cast<double *>(static_cast<unsigned long long *>(base) + NOALLOC_PARTIALS)};
    hipStream_t s = (hipStream_t)stream;
    PX_HIP(relax_launch(dtype, a, s), "relax kernel launch");
    if (resmode != RES_NONE) PX_HIP(reduce_partials(a.part, parts, norms, s), "norm reduction launch");
    return PX_OK;
}

int px_autotune(const void *phi_in, void *phi_out, int n, int ld, int dtype, const void *f, int ld_f,
                int bc, px_ctx *ctx, void *stream, int *best_k, int *best_rows, double *gcells)
{
    int st = check_n_ld(n, ld, dtype);
    if (st) return st;
    if ((st = check_ptr(phi_in, dtype, "phi_in")) || (st = check_ptr(phi_out, dtype, "phi_out")))
        return st;
    if ((st = check_flat(f, n, ld_f, dtype, "f"))) return st;
    if (!valid_bc(bc)) return fail(PX_EINVAL, "unknown bc %d", bc);
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    const size_t gb = grid_bytes(n, ld, dtype);
    if (overlap(phi_in, gb, phi_out, gb)) return fail(PX_EALIAS, "phi_out overlaps phi_in");
    if (overlap(f, flat_bytes(n, ld_f, dtype), phi_out, gb)) return fail(PX_EALIAS, "phi_out overlaps f");
    if ((st = set_device(ctx))) return st;
    hipStream_t s = (hipStream_t)stream;
    // Candidate tile heights: short bands give more waves, long bands less halo
    // recomputation; the best also depends on how the wave count divides the
    // resident wave slots, so the list is dense.
    static const int ROWS[] = {4, 6, 8, 12, 16, 20, 24, 28, 29, 32, 36, 38, 40, 44, 47, 48, 56, 64, 80, 96, 128};
    const double h = 1.0 / n, lambda = 0.25 * h * h * (2.0 / 3.0);
    hipEvent_t e0, e1;
    PX_HIP(hipEventCreate(&e0), "hipEventCreate");
    PX_HIP(hipEventCreate(&e1), "hipEventCreate");
    // first pass: every candidate, fastest of five single launches; the TOP best go on
    // to a second pass of back-to-back launches (the way a sweep loop runs them), which
    // separates candidates that single launches rank within their noise
    constexpr int TOP = 4;
    struct Cand { double g; int k, rows; };
    Cand top[TOP] = {};
    int err = PX_OK;
    for (int k = 1; k <= 8 && !err; ++k) {
        int last = -1;
        for (int rows : ROWS) {
            // with k + 1 a multiple of 3 the unrolled loop runs blocks of k + 1 row steps: from
            // 16 rows up, take the next height that fills its last block (rows + 2k a multiple
            // of k + 1), whose partial block would otherwise compute rows it never stores
            if ((k + 1) % 3 == 0 && rows >= 16) rows += ((k + 1) - (rows + 2 * k) % (k + 1)) % (k + 1);
            if (rows == last) continue;
            last = rows;
            if (rows > std::max(8, n + 2)) break;
            // one warm-up launch of k sweeps, then the fastest of five individually timed
            // launches (the minimum is robust against clock ramps and interference)
            if ((err = run_sweeps(ctx, dtype, phi_in, phi_out, nullptr, n, ld, f, ld_f, h, lambda, k, k, bc,
                                  RES_NONE, nullptr, s, rows)))
                break;
            float ms = 0.f;
            for (int rep = 0; rep < 5 && !err; ++rep) {
                hipError_t he = hipEventRecord(e0, s);
                if (he == hipSuccess)
                    err = run_sweeps(ctx, dtype, phi_in, phi_out, nullptr, n, ld, f, ld_f, h, lambda, k, k, bc,
                                     RES_NONE, nullptr, s, rows);
                if (err) break;
                if (he == hipSuccess) he = hipEventRecord(e1, s);
                if (he == hipSuccess) he = hipEventSynchronize(e1);
                float one = 0.f;
                if (he == hipSuccess) he = hipEventElapsedTime(&one, e0, e1);
                if (he != hipSuccess) {
                    err = hip_fail(he, "autotune timing");
                    break;
                }
                if (rep == 0 || one < ms) ms = one;
            }
            if (err) break;
            const double g = ms > 0.f ? k * (double)n * n / (ms * 1e-3) / 1e9 : 0.0;
            for (int i = 0; i < TOP; ++i) {
                if (g > top[i].g) {
                    for (int j = TOP - 1; j > i; --j) top[j] = top[j - 1];
                    top[i] = Cand{g, k, rows};
                    break;
                }
            }
        }
    }
    // Second pass: runs of RUN launches as a sweep loop makes them -- each launch reading
    // the previous one's output, alternating between phi_out and the context's grid -- so
    // that what the caches hold between launches is what a real run sees (single launches
    // re-read the same input, which the Infinity Cache may still hold, and rank tile
    // heights differently).
    constexpr int RUN = 24, ROUNDS = 3;  // runs as long as a 200-sweep call at k = 8
    if (!err) err = ensure_grid(ctx, gb);
    double g2[TOP] = {};
    for (int round = 0; round < ROUNDS && !err; ++round) {
        for (int i = 0; i < TOP && !err; ++i) {
            if (top[i].k == 0) continue;
            hipError_t he = hipEventRecord(e0, s);
            if (he == hipSuccess)
                err = run_sweeps(ctx, dtype, phi_in, phi_out, ctx->grid, n, ld, f, ld_f, h, lambda, RUN * top[i].k,
                                 top[i].k, bc, RES_NONE, nullptr, s, top[i].rows);
            if (err) break;
            if (he == hipSuccess) he = hipEventRecord(e1, s);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            float ms = 0.f;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess) {
                err = hip_fail(he, "autotune timing");
                break;
            }
            const double g = ms > 0.f ? RUN * top[i].k * (double)n * n / (ms * 1e-3) / 1e9 : 0.0;
            g2[i] = std::max(g2[i], g);
        }
    }
    // the two best of the second pass go on
    int order[TOP];
    for (int i = 0; i < TOP; ++i) order[i] = i;
    std::sort(order, order + TOP, [&](int a, int b) { return g2[a] > g2[b]; });
    constexpr int FIN = 2;
    int rn[FIN] = {0, 0};
    // third pass: for each, the tile height of its launches that also take the norms (their
    // pipeline holds one more level, the residual's, so they favour other heights): the
    // fastest of three single launches per height
    if (!err) err = ensure_norms(ctx);
    for (int c = 0; c < FIN && !err; ++c) {
        const int kc = top[order[c]].k;
        if (kc == 0) continue;
        if (c == 1 && kc == top[order[0]].k) {
            rn[1] = rn[0];
            continue;
        }
        float best_norm = 0.f;
        for (int rows : ROWS) {
            if (err || rows > std::max(8, n + 2)) break;
            if ((err = run_sweeps(ctx, dtype, phi_in, phi_out, nullptr, n, ld, f, ld_f, h, lambda, kc, kc, bc,
                                  RES_FINAL, ctx->norms_dev, s, rows)))
                break;
            for (int rep = 0; rep < 3 && !err; ++rep) {
                hipError_t he = hipEventRecord(e0, s);
                if (he == hipSuccess)
                    err = run_sweeps(ctx, dtype, phi_in, phi_out, nullptr, n, ld, f, ld_f, h, lambda, kc, kc, bc,
                                     RES_FINAL, ctx->norms_dev, s, rows);
                if (err) break;
                if (he == hipSuccess) he = hipEventRecord(e1, s);
                if (he == hipSuccess) he = hipEventSynchronize(e1);
                float one = 0.f;
                if (he == hipSuccess) he = hipEventElapsedTime(&one, e0, e1);
                if (he != hipSuccess) {
                    err = hip_fail(he, "autotune timing");
                    break;
                }
                if (rn[c] == 0 || one < best_norm) {
                    best_norm = one;
                    rn[c] = rows;
                }
            }
        }
    }
    // final pass: each as a whole call makes it -- RUN launches from phi_in, each reading
    // the previous output, the last one also taking the norms at its own height -- the
    // median of five alternating calls (a sweep loop runs at its typical, not its best,
    // rate: the fastest of a few calls had favoured shorter bands that run slower on
    // average)
    constexpr int FROUNDS = 5;
    double g5[FIN][FROUNDS] = {};
    for (int round = 0; round < FROUNDS && !err; ++round) {
        for (int c = 0; c < FIN && !err; ++c) {
            const Cand &cd = top[order[c]];
            if (cd.k == 0) continue;
            hipError_t he = hipEventRecord(e0, s);
            if (he == hipSuccess)
                err = run_sweeps(ctx, dtype, phi_in, phi_out, ctx->grid, n, ld, f, ld_f, h, lambda, RUN * cd.k, cd.k,
                                 bc, RES_FINAL, ctx->norms_dev, s, cd.rows, rn[c]);
            if (err) break;
            if (he == hipSuccess) he = hipEventRecord(e1, s);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            float ms = 0.f;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess) {
                err = hip_fail(he, "autotune timing");
                break;
            }
            g5[c][round] = ms > 0.f ? RUN * cd.k * (double)n * n / (ms * 1e-3) / 1e9 : 0.0;
        }
    }
    double g4[FIN] = {0.0, 0.0};
    for (int c = 0; c < FIN; ++c) {
        std::sort(g5[c], g5[c] + FROUNDS);
        g4[c] = g5[c][FROUNDS / 2];
    }
    // within 1.5% of each other the taller band wins at equal k: it recomputes fewer halo
    // rows and reads less, and in long sweep loops (clocks settled, the memory system
    // loaded) it has held up better than the timing of a few calls shows
    int win = (g4[1] > g4[0]) ? 1 : 0;
    {
        const Cand &a = top[order[0]], &b = top[order[1]];
        if (a.k == b.k && b.k != 0 && std::max(g4[0], g4[1]) <= 1.015 * std::min(g4[0], g4[1]))
            win = (b.rows > a.rows) ? 1 : 0;
    }
    const int bk = top[order[win]].k, br = top[order[win]].rows, brn = rn[win];
    const double bg = g4[win];
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err) return err;
    px_tuned &t = ctx->tuned[dtype];
    t.rows_norm = brn;
    t.n = n;
    t.ld = ld;
    t.k = bk;
    t.rows = br;
    t.gcells = bg;
    if (best_k) *best_k = bk;
    if (best_rows) *best_rows = br;
    if (gcells) *gcells = bg;
    return PX_OK;
}

// Default sweeps per inner solve of the mixed modes.  Long inner solves amortise the FP64
// step (at 8192^2: 24 us per FP32 sweep with 1024 per step, 32 us with 64).  Each sweep
// rounds the correction d to the storage type; after m sweeps d holds about m * lambda
// times the residual, so the rounding leaves a high-frequency residual of about
// eps * (8 / h^2) * m * lambda = 2 * omega * eps * m times |r| (eps = 2^-24 FP32, 2^-9
// BF16).  Refinement converges while that stays below 1: FP32 with m = 1024 is at 1e-4
// and takes exactly the sweeps of plain FP64; BF16 (an 8-bit significand) stalls near
// m = 1024 and gets m = 128 (0.33).  The same for every grid size, so a batch and its
// members solved one by one take the same steps; a solve stops at the end of the step
// that reaches the tolerance.
static int default_inner(int mode) { return mode == PX_SOLVE_MIXED_F32 ? 1024 : 128; }

int px_solve(void *phi, int n, int ld, int dtype, const void *f, int ld_f, double h, double lambda,
             const px_solve_opts *o, px_solve_stats *stats, px_ctx *ctx, void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    int st = check_n_ld(n, ld, dtype);
    if (st) return st;
    if (!o) return fail(PX_EINVAL, "opts is NULL");
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    if ((st = check_ptr(phi, dtype, "phi"))) return st;
    if ((st = check_flat(f, n, ld_f, dtype, "f"))) return st;
    if ((st = check_pos(h, "h")) || (st = check_pos(lambda, "lambda"))) return st;
    if (o->mode < PX_SOLVE_PLAIN || o->mode > PX_SOLVE_MIXED_BF16) return fail(PX_EINVAL, "unknown mode %d", o->mode);
    if (o->mode != PX_SOLVE_PLAIN && dtype != F64)
        return fail(PX_EINVAL, "mixed-precision modes need FP64 phi and f");
    if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol)) return fail(PX_EINVAL, "rtol must be finite and >= 0");
    if (o->norm != 0 && o->norm != 1) return fail(PX_EINVAL, "norm must be 0 (max) or 1 (L2)");
    if (o->max_sweeps < 0) return fail(PX_EINVAL, "max_sweeps < 0");
    if (o->tblock < 0 || o->tblock > 8) return fail(PX_EINVAL, "tblock outside [0, 8]");
    if (!valid_bc(o->bc)) return fail(PX_EINVAL, "unknown bc %d", o->bc);
    if (o->bc == PERIODIC && o->mode != PX_SOLVE_PLAIN)
        return fail(PX_EUNSUPPORTED, "mixed-precision refinement takes the Dirichlet and fixed-ghost boundaries");
    const int check_every = o->check_every > 0 ? o->check_every : 100;
    const int inner = o->inner_sweeps > 0 ? o->inner_sweeps : default_inner(o->mode);
    const size_t gb = grid_bytes(n, ld, dtype);
    if (overlap(f, flat_bytes(n, ld_f, dtype), phi, gb)) return fail(PX_EALIAS, "phi overlaps f");
    if ((st = set_device(ctx))) return st;
    if ((st = ensure_norms(ctx))) return st;
    if ((st = ensure_grid(ctx, gb))) return st;
    hipStream_t s = (hipStream_t)stream;
    const int bc = o->bc;
    const int k = o->tblock ? o->tblock : default_tblock(ctx, dtype, n, ld);

    auto read_norms = [&](double *dst) -> int {
        PX_HIP(hipMemcpyAsync(ctx->norms_host, ctx->norms_dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s),
               "norm readback");
        PX_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        dst[0] = ctx->norms_host[0];
        dst[1] = ctx->norms_host[1];
        return PX_OK;
    };
    auto measure = [&](const double *nr) { return o->norm == 0 ? nr[0] : std::sqrt(nr[1]); };

    // norms of f: the residual of the zero iterate is f itself
    double fn[2];
    {
        // residual of zero: use the ctx grid, zeroed, as phi
        PX_HIP(zero_grid_launch(dtype, ctx->grid, n, ld, s), "zero kernel launch");
        if ((st = residual_into(ctx, dtype, ctx->grid, n, ld, f, ld_f, h, GHOST_FIXED, nullptr, 0,
                                ctx->norms_dev, s)))
            return st;
        if ((st = read_norms(fn))) return st;
    }
    const double fref = measure(fn);
    const double target = o->rtol * fref;

    px_solve_stats S;
    std::memset(&S, 0, sizeof S);
    double nr[2] = {0, 0};
    int result = PX_OK;
    void *cur = phi;
    void *oth = ctx->grid;

    if (o->mode == PX_SOLVE_PLAIN) {
        if ((st = residual_into(ctx, dtype, phi, n, ld, f, ld_f, h, bc, nullptr, 0, ctx->norms_dev, s)))
            return st;
        if ((st = read_norms(nr))) return st;
        const double r0 = measure(nr);
        for (;;) {
            const double m = measure(nr);
            if (!std::isfinite(nr[0]) || !std::isfinite(nr[1])) { result = fail(PX_ENONFINITE, "non-finite residual"); break; }
            if (m <= target) break;
            if (m > 1e8 * std::max(r0, fref)) { result = fail(PX_EDIVERGED, "residual grew from %g to %g", r0, m); break; }
            if (S.sweeps >= o->max_sweeps) { result = fail(PX_ENOTCONV, "max_sweeps reached (rel res %g)", m / fref); break; }
            const int todo = (int)std::min<int64_t>(check_every, o->max_sweeps - S.sweeps);
            // one launch sequence cur -> oth; intermediate launches alternate through cur itself
            // is not allowed (cur is the source), so run them as single-launch chunks of k.
            int done = 0;
            while (done < todo) {
                const int ks = std::min(k, todo - done);
                const bool last = done + ks == todo;
                if ((st = run_sweeps(ctx, dtype, cur, oth, nullptr, n, ld, f, ld_f, h, lambda, ks, ks, bc,
                                     last ? RES_FINAL : RES_NONE, ctx->norms_dev, s)))
                    return st;
                std::swap(cur, oth);
                done += ks;
            }
            S.sweeps += todo;
            S.outer_steps += 1;
            if ((st = read_norms(nr))) return st;
        }
        if (cur != phi) PX_HIP(copy_grid_launch(dtype, cur, phi, n, ld, s), "copy kernel launch");
    } else {
        const int lowp = (o->mode == PX_SOLVE_MIXED_F32) ? F32 : BF16;
        // low-precision grids: rows padded to 128 bytes (the pitch of grids the caller
        // allocates the same way, so an autotuned configuration for it applies)
        const int per_line = 128 / elem_size(lowp);
        const int ldl = (n + 2 + per_line - 1) / per_line * per_line;
        const int k_in = o->tblock ? o->tblock : default_tblock(ctx, lowp, n, ldl);
        // Grids up to 1024^2 are launch-bound: there the solve runs as a batch of one,
        // whose outer steps are replayed from a captured graph with the convergence test on
        // the device (same arithmetic and stopping rules, identical results).  It needs rows
        // of phi and f on 16-byte boundaries.
        const bool graph_ok = n <= 1024 && reinterpret_cast<uintptr_t>(phi) % 16 == 0 &&
                              reinterpret_cast<uintptr_t>(f) % 16 == 0 && (ld * 8) % 16 == 0 &&
                              (ld_f * 8) % 16 == 0;
        if (graph_ok) {
            if (!ctx->batch) ctx->batch = new (std::nothrow) BatchWork();
            if (!ctx->batch) return fail(PX_ENOMEM, "out of host memory");
            BatchProblem bp{phi, f, n, ld, ld_f, h, lambda};
            BatchStat bs;
            char err[256] = "";
            const int ks = std::min(k_in, inner);
            st = batch_solve(*ctx->batch, lowp, &bp, 1, bc, o->rtol, o->norm, o->max_sweeps, inner, ks, 8,
                             pick_rows(ctx, lowp, n, ldl, ks), &bs, s, err, sizeof err);
            // a problem that did not converge is reported through bs.state below
            if (st != PX_OK && st != PX_ENOTCONV && st != PX_ENONFINITE && st != PX_EDIVERGED)
                return fail(st, "%s", err);
            S.sweeps = bs.sweeps;
            S.outer_steps = bs.steps;
            S.res_max = bs.res_max;
            S.res_l2 = bs.res_l2;
            S.rel_res_max = bs.rel_res_max;
            S.rel_res_l2 = bs.rel_res_l2;
            S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (stats) *stats = S;
            switch (bs.state) {
            case 0: return PX_OK;
            case -1: return fail(PX_ENOTCONV, "max_sweeps reached (rel res %g)", o->norm ? bs.rel_res_l2 : bs.rel_res_max);
            case -2: return fail(PX_ENONFINITE, "non-finite residual");
            default: return fail(PX_EDIVERGED, "residual grew beyond 1e8 times its start");
            }
        }
        // host readbacks every `spacing` outer steps (the device computes norms every step)
        const int spacing = o->check_every > inner ? o->check_every / inner : 1;
        const size_t lg = grid_bytes(n, ldl, lowp);
        const size_t lr = flat_bytes(n, ldl, lowp);
        // three ghosted low-precision grids (zero start, ping, pong) and r_low
        const size_t gsz = (lg + 255) / 256 * 256;
        const size_t off_r = 3 * gsz;
        if ((st = ensure_mix(ctx, off_r + (lr + 255) / 256 * 256))) return st;
        char *mb = static_cast<char *>(ctx->mix);
        void *da = mb, *db = mb + gsz, *dc = mb + 2 * gsz;
        void *rl = mb + off_r;  // 256-byte aligned, rows of ldl elements: vector loads
        const int nblk = pointwise_num_blocks(n);
        if ((st = ensure_partials(ctx, (size_t)nblk))) return st;
        // step 0: oth = phi (copy with ghosts per bc), r = f - L phi
        PX_HIP(refine_launch(lowp, (const double *)cur, nullptr, 0, (double *)oth, n, ld, (const double *)f,
                             ld_f, 1.0 / (h * h), bc, rl, ldl, partials(ctx), s),
               "refine kernel launch");
        PX_HIP(reduce_partials(partials(ctx), nblk, ctx->norms_dev, s), "norm reduction launch");
        std::swap(cur, oth);
        if ((st = read_norms(nr))) return st;
        const double r0 = measure(nr);
        for (;;) {
            const double m = measure(nr);
            if (!std::isfinite(nr[0]) || !std::isfinite(nr[1])) { result = fail(PX_ENONFINITE, "non-finite residual"); break; }
            if (m <= target) break;
            if (m > 1e8 * std::max(r0, fref)) { result = fail(PX_EDIVERGED, "residual grew from %g to %g", r0, m); break; }
            if (S.sweeps >= o->max_sweeps) { result = fail(PX_ENOTCONV, "max_sweeps reached (rel res %g)", m / fref); break; }
            // inner: delta = 0, `inner` low-precision sweeps on L delta = r_low
            PX_HIP(zero_grid_launch(lowp, da, n, ldl, s), "zero kernel launch");
            if ((st = run_sweeps(ctx, lowp, da, db, dc, n, ldl, rl, ldl, h, lambda, inner,
                                 std::min(k_in, inner), bc, RES_NONE, nullptr, s)))
                return st;
            // outer: oth = cur + delta (FP64), r = f - L oth
            PX_HIP(refine_launch(lowp, (const double *)cur, db, ldl, (double *)oth, n, ld, (const double *)f, ld_f,
                                 1.0 / (h * h), bc, rl, ldl, partials(ctx), s),
                   "refine kernel launch");
            PX_HIP(reduce_partials(partials(ctx), nblk, ctx->norms_dev, s), "norm reduction launch");
            std::swap(cur, oth);
            S.sweeps += inner;
            S.outer_steps += 1;
            if (S.outer_steps % spacing == 0 || S.sweeps >= o->max_sweeps)
                if ((st = read_norms(nr))) return st;
        }
        if (cur != phi) PX_HIP(copy_grid_launch(dtype, cur, phi, n, ld, s), "copy kernel launch");
    }
    PX_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    S.res_max = nr[0];
    S.res_l2 = std::sqrt(nr[1]);
    S.rel_res_max = fn[0] > 0 ? nr[0] / fn[0] : nr[0];
    S.rel_res_l2 = fn[1] > 0 ? std::sqrt(nr[1] / fn[1]) : S.res_l2;
    S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = S;
    return result;
}

static int check_batch(const px_problem *probs, int nprob, int dtype, std::vector<BatchProblem> &out)
{
    if (!probs) return fail(PX_EINVAL, "probs is NULL");
    if (nprob < 1 || nprob > (1 << 20)) return fail(PX_EINVAL, "nprob = %d outside [1, 2^20]", nprob);
    if (!valid_dtype(dtype)) return fail(PX_EINVAL, "unknown dtype %d", dtype);
    const size_t es = (size_t)elem_size(dtype);
    out.resize(nprob);
    std::vector<std::pair<uintptr_t, uintptr_t>> ranges(nprob);
    for (int p = 0; p < nprob; ++p) {
        const px_problem &q = probs[p];
        int st = check_n_ld(q.n, q.ld, dtype);
        if (!st) st = check_ptr(q.phi, dtype, "phi");
        if (!st) st = check_flat(q.f, q.n, q.ld_f, dtype, "f");
        if (!st) st = check_pos(q.h, "h");
        if (!st) st = check_pos(q.lambda, "lambda");
        if (st) return fail(st, "problem %d: %s", p, px_last_error());
        if (reinterpret_cast<uintptr_t>(q.phi) % 16 || reinterpret_cast<uintptr_t>(q.f) % 16 ||
            ((size_t)q.ld * es) % 16 || ((size_t)q.ld_f * es) % 16)
            return fail(PX_EINVAL, "problem %d: rows of phi and f must start on 16-byte boundaries", p);
        const size_t gb = grid_bytes(q.n, q.ld, dtype);
        if (overlap(q.f, flat_bytes(q.n, q.ld_f, dtype), q.phi, gb))
            return fail(PX_EALIAS, "problem %d: phi overlaps f", p);
        ranges[p] = {reinterpret_cast<uintptr_t>(q.phi), reinterpret_cast<uintptr_t>(q.phi) + gb};
        out[p] = BatchProblem{q.phi, q.f, q.n, q.ld, q.ld_f, q.h, q.lambda};
    }
    std::sort(ranges.begin(), ranges.end());
    for (int p = 1; p < nprob; ++p)
        if (ranges[p].first < ranges[p - 1].second) return fail(PX_EALIAS, "two problems' phi overlap");
    return PX_OK;
}

int px_relax_batched(const px_problem *probs, int nprob, int dtype, int nsweeps, int tblock, int bc,
                     int resmode, double *norms, px_ctx *ctx, void *stream)
{
    std::vector<BatchProblem> bp;
    int st = check_batch(probs, nprob, dtype, bp);
    if (st) return st;
    if (nsweeps < 1) return fail(PX_EINVAL, "nsweeps = %d < 1", nsweeps);
    if (tblock < 0 || tblock > 8) return fail(PX_EINVAL, "tblock = %d outside [0, 8]", tblock);
    if (!valid_bc(bc)) return fail(PX_EINVAL, "unknown bc %d", bc);
    if (bc == PERIODIC) return fail(PX_EUNSUPPORTED, "batches take the Dirichlet and fixed-ghost boundaries");
    if (resmode < RES_NONE || resmode > RES_FINAL) return fail(PX_EINVAL, "unknown resmode %d", resmode);
    if (resmode == RES_LAGGED) return fail(PX_EUNSUPPORTED, "batched relaxation reports FINAL norms only");
    if (resmode == RES_FINAL && !norms) return fail(PX_EINVAL, "norms is NULL");
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    if ((st = set_device(ctx))) return st;
    if (!ctx->batch) ctx->batch = new (std::nothrow) BatchWork();
    if (!ctx->batch) return fail(PX_ENOMEM, "out of host memory");
    char err[256] = "";
    const int tk = ctx->batch->tuned_k[dtype];
    st = batch_relax(*ctx->batch, dtype, bp.data(), nprob, nsweeps, tblock ? tblock : (tk ? tk : 8), bc, resmode,
                     norms, ctx->tile_rows, (hipStream_t)stream, err, sizeof err);
    return st ? fail(st, "%s", err) : PX_OK;
}

int px_relax_boxes(const px_problem *boxes, int nbx, int nby, int dtype, int nsweeps, int exchange, int bc,
                   px_ctx *ctx, void *stream)
{
    if (nbx < 1 || nby < 1 || (long long)nbx * nby > 65535)
        return fail(PX_EINVAL, "box layout %d x %d outside 1..65535 boxes", nbx, nby);
    std::vector<BatchProblem> bp;
    int st = check_batch(boxes, nbx * nby, dtype, bp);
    if (st) return st;
    for (int b = 1; b < nbx * nby; ++b)
        if (bp[b].n != bp[0].n || bp[b].h != bp[0].h || bp[b].lambda != bp[0].lambda)
            return fail(PX_EINVAL, "box %d: every box of a domain needs the same n, h and lambda", b);
    if (nsweeps < 0) return fail(PX_EINVAL, "nsweeps = %d < 0", nsweeps);
    if (exchange < 1 || exchange > 8) return fail(PX_EINVAL, "exchange = %d outside [1, 8]", exchange);
    if (nsweeps % exchange) return fail(PX_EINVAL, "nsweeps = %d is not a multiple of exchange = %d", nsweeps, exchange);
    if (!valid_bc(bc)) return fail(PX_EINVAL, "unknown bc %d", bc);
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    if ((st = set_device(ctx))) return st;
    if (!ctx->batch) ctx->batch = new (std::nothrow) BatchWork();
    if (!ctx->batch) return fail(PX_ENOMEM, "out of host memory");
    char err[256] = "";
    st = batch_relax_boxes(*ctx->batch, dtype, bp.data(), nbx, nby, nsweeps, exchange, bc, ctx->tile_rows,
                           (hipStream_t)stream, err, sizeof err);
    return st ? fail(st, "%s", err) : PX_OK;
}

int px_autotune_batched(const px_problem *probs, int nprob, int dtype, int bc, px_ctx *ctx, void *stream, int *best_k)
{
    std::vector<BatchProblem> bp;
    int st = check_batch(probs, nprob, dtype, bp);
    if (st) return st;
    if (!valid_bc(bc)) return fail(PX_EINVAL, "unknown bc %d", bc);
    if (bc == PERIODIC) return fail(PX_EUNSUPPORTED, "batches take the Dirichlet and fixed-ghost boundaries");
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    if ((st = set_device(ctx))) return st;
    if (!ctx->batch) ctx->batch = new (std::nothrow) BatchWork();
    if (!ctx->batch) return fail(PX_ENOMEM, "out of host memory");
    char err[256] = "";
    st = batch_autotune(*ctx->batch, dtype, bp.data(), nprob, bc, (hipStream_t)stream, best_k, err, sizeof err);
    return st ? fail(st, "%s", err) : PX_OK;
}

int px_solve_batched(const px_problem *probs, int nprob, const px_solve_opts *o, px_solve_stats *stats,
                     px_ctx *ctx, void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<BatchProblem> bp;
    int st = check_batch(probs, nprob, F64, bp);
    if (st) return st;
    if (!o) return fail(PX_EINVAL, "opts is NULL");
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    if (o->mode == PX_SOLVE_PLAIN) return fail(PX_EUNSUPPORTED, "batched solves refine around FP32/BF16 sweeps");
    if (o->mode != PX_SOLVE_MIXED_F32 && o->mode != PX_SOLVE_MIXED_BF16) return fail(PX_EINVAL, "unknown mode");
    if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol)) return fail(PX_EINVAL, "rtol must be finite and >= 0");
    if (o->norm != 0 && o->norm != 1) return fail(PX_EINVAL, "norm must be 0 (max) or 1 (L2)");
    if (o->max_sweeps < 0) return fail(PX_EINVAL, "max_sweeps < 0");
    if (o->tblock < 0 || o->tblock > 8) return fail(PX_EINVAL, "tblock outside [0, 8]");
    if (!valid_bc(o->bc)) return fail(PX_EINVAL, "unknown bc %d", o->bc);
    if (o->bc == PERIODIC) return fail(PX_EUNSUPPORTED, "batches take the Dirichlet and fixed-ghost boundaries");
    const int inner = o->inner_sweeps > 0 ? o->inner_sweeps : default_inner(o->mode);
    if ((st = set_device(ctx))) return st;
    if (!ctx->batch) ctx->batch = new (std::nothrow) BatchWork();
    if (!ctx->batch) return fail(PX_ENOMEM, "out of host memory");
    std::vector<BatchStat> bs(nprob);
    char err[256] = "";
    const int lowp = o->mode == PX_SOLVE_MIXED_F32 ? F32 : BF16;
    const int tk = ctx->batch->tuned_k[lowp];
    const int k = std::min(o->tblock ? o->tblock : (tk ? tk : 8), inner);
    st = batch_solve(*ctx->batch, lowp, bp.data(), nprob, o->bc, o->rtol, o->norm, o->max_sweeps, inner, k, 8,
                     ctx->tile_rows,
                     bs.data(), (hipStream_t)stream, err, sizeof err);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats)
        for (int p = 0; p < nprob; ++p) {
            px_solve_stats &S = stats[p];
            S.sweeps = bs[p].sweeps;
            S.outer_steps = bs[p].steps;
            S.res_max = bs[p].res_max;
            S.res_l2 = bs[p].res_l2;
            S.rel_res_max = bs[p].rel_res_max;
            S.rel_res_l2 = bs[p].rel_res_l2;
            S.seconds = secs;
        }
    return st ? fail(st, "%s", err) : PX_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- learned correction

extern "C" {

int px_net_make_pair(const double *phi, int n, int ld, int loss, float *x, float *t, px_ctx *ctx, void *stream)
{
    int st = check_n_ld(n, ld, F64);
    if (st) return st;
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    if ((st = check_ptr(phi, F64, "phi"))) return st;
    if (!x || !t) return fail(PX_EINVAL, "x or t is NULL");
    if (loss != PX_LOSS_MSE && loss != PX_LOSS_ENERGY) return fail(PX_EINVAL, "unknown loss %d", loss);
    const size_t gb = grid_bytes(n, ld, F64), xb = sizeof(float) * (size_t)n * n;
    if (overlap(x, xb, phi, gb) || overlap(t, xb, phi, gb) || overlap(x, xb, t, xb))
        return fail(PX_EALIAS, "x, t and phi must not overlap");
    if ((st = set_device(ctx))) return st;
    const size_t pb = sizeof(double) * 2 * (size_t)pair_num_blocks(n);
    if ((st = ensure_mix(ctx, pb + 2 * sizeof(double)))) return st;
    double *part = static_cast<double *>(ctx->mix);
    PX_HIP(pair_launch(phi, n, ld, loss, x, t, part, part + pb / sizeof(double), (hipStream_t)stream),
           "pair kernel launch");
    return PX_OK;
}

int px_correction_step(void *phi, int n, int ld, const double *r, int ld_r, const void *d, int d_dtype, int ld_d,
                       double h, int mode, double *coef, px_ctx *ctx, void *stream)
{
    int st = check_n_ld(n, ld, F64);
    if (st) return st;
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    if ((st = check_ptr(phi, F64, "phi"))) return st;
    if ((st = check_flat(r, n, ld_r, F64, "r"))) return st;
    if (mode < 0 || mode > 2) return fail(PX_EINVAL, "mode must be 0, 1 or 2");
    if (!d) {
        if (mode != 0) return fail(PX_EINVAL, "d is NULL");
        d = r;
        d_dtype = F64;
        ld_d = ld_r;
    }
    if (d_dtype != F64 && d_dtype != F32) return fail(PX_EINVAL, "d_dtype must be PX_F64 or PX_F32");
    if ((st = check_flat(d, n, ld_d, d_dtype, "d"))) return st;
    if ((st = check_pos(h, "h"))) return st;
    const size_t gb = grid_bytes(n, ld, F64);
    if (overlap(phi, gb, r, flat_bytes(n, ld_r, F64)) || overlap(phi, gb, d, flat_bytes(n, ld_d, d_dtype)))
        return fail(PX_EALIAS, "phi overlaps r or d");
    if ((st = set_device(ctx))) return st;
    const size_t pb = sizeof(double) * 8 * (size_t)pair_num_blocks(n);
    if ((st = ensure_mix(ctx, pb + 8 * sizeof(double)))) return st;
    double *part = static_cast<double *>(ctx->mix);
    PX_HIP(correction_launch(d_dtype, d, ld_d, r, ld_r, static_cast<double *>(phi), n, ld, 1.0 / (h * h), mode, part,
                             part + pb / sizeof(double), coef, (hipStream_t)stream),
           "correction step launch");
    return PX_OK;
}

int px_solve_learned(void *phi, int n, int ld, const double *f, int ld_f, double h, double lambda, px_net *net,
                     const px_learned_opts *o, px_learned_stats *stats, px_ctx *ctx, void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    int st = check_n_ld(n, ld, F64);
    if (st) return st;
    if (!o) return fail(PX_EINVAL, "opts is NULL");
    if (!ctx) return fail(PX_EINVAL, "ctx is NULL");
    if ((st = check_ptr(phi, F64, "phi"))) return st;
    if ((st = check_flat(f, n, ld_f, F64, "f"))) return st;
    if ((st = check_pos(h, "h")) || (st = check_pos(lambda, "lambda"))) return st;
    if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol)) return fail(PX_EINVAL, "rtol must be finite and >= 0");
    if (o->norm != 0 && o->norm != 1) return fail(PX_EINVAL, "norm must be 0 (max) or 1 (L2)");
    if (o->max_sweeps < 0) return fail(PX_EINVAL, "max_sweeps < 0");
    if (o->smooth_sweeps < 1) return fail(PX_EINVAL, "smooth_sweeps must be >= 1");
    if (o->tblock < 0 || o->tblock > 8) return fail(PX_EINVAL, "tblock outside [0, 8]");
    if (o->use_net < 0 || o->use_net > 2) return fail(PX_EINVAL, "use_net must be 0, 1 or 2");
    if (o->judge < 0 || o->judge > 2) return fail(PX_EINVAL, "judge must be 0, 1 or 2");
    if (o->use_net && !net) return fail(PX_EINVAL, "use_net needs a network");
    if (o->use_net && net_device(net) != ctx->device)
        return fail(PX_EINVAL, "network on device %d, context on device %d", net_device(net), ctx->device);
    const size_t gb = grid_bytes(n, ld, F64);
    if (overlap(f, flat_bytes(n, ld_f, F64), phi, gb)) return fail(PX_EALIAS, "phi overlaps f");
    if ((st = set_device(ctx))) return st;
    if ((st = ensure_norms(ctx))) return st;
    if ((st = ensure_grid(ctx, gb))) return st;
    // scratch: saved iterate | r (FP64) | network output (FP32) | double2 partials | dots
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const int ld_r = (n + 31) / 32 * 32, ld_y = (n + 63) / 64 * 64;
    const size_t o_r = up(gb), o_y = o_r + up(sizeof(double) * (size_t)n * ld_r);
    const size_t o_p = o_y + up(sizeof(float) * (size_t)n * ld_y);
    const size_t o_d = o_p + up(sizeof(double) * 8 * (size_t)pair_num_blocks(n));
    if ((st = ensure_mix(ctx, o_d + 256))) return st;
    char *mb = static_cast<char *>(ctx->mix);
    double *save = reinterpret_cast<double *>(mb);
    double *r = reinterpret_cast<double *>(mb + o_r);
    float *y = reinterpret_cast<float *>(mb + o_y);
    double *part = reinterpret_cast<double *>(mb + o_p);
    double *dots = reinterpret_cast<double *>(mb + o_d);
    hipStream_t s = (hipStream_t)stream;
    const int k = o->tblock ? o->tblock : default_tblock(ctx, F64, n, ld);
    const double c = 1.0 / (h * h);

    auto read_norms = [&](double *dst) -> int {
        PX_HIP(hipMemcpyAsync(ctx->norms_host, ctx->norms_dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s),
               "norm readback");
        PX_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
        dst[0] = ctx->norms_host[0];
        dst[1] = ctx->norms_host[1];
        return PX_OK;
    };
    auto measure = [&](const double *nr) { return o->norm == 0 ? nr[0] : std::sqrt(nr[1]); };

    double fn[2];
    PX_HIP(zero_grid_launch(F64, ctx->grid, n, ld, s), "zero kernel launch");
    if ((st = residual_into(ctx, F64, ctx->grid, n, ld, f, ld_f, h, GHOST_FIXED, nullptr, 0, ctx->norms_dev, s)))
        return st;
    if ((st = read_norms(fn))) return st;
    const double fref = measure(fn);
    const double target = o->rtol * fref;

    px_learned_stats S;
    std::memset(&S, 0, sizeof S);
    double nr[2] = {0, 0};
    int result = PX_OK;
    void *cur = phi;
    void *oth = ctx->grid;
    bool correct = true;

    // sweeps cur -> ... in single-launch chunks of k (cur ends on the last output)
    auto smooth = [&](int todo, bool norms_at_end) -> int {
        int done = 0;
        while (done < todo) {
            const int ks = std::min(k, todo - done);
            const bool last = done + ks == todo;
            int e = run_sweeps(ctx, F64, cur, oth, nullptr, n, ld, f, ld_f, h, lambda, ks, ks, DIRICHLET0,
                               (last && norms_at_end) ? RES_FINAL : RES_NONE, ctx->norms_dev, s);
            if (e) return e;
            std::swap(cur, oth);
            done += ks;
        }
        return PX_OK;
    };

    if ((st = residual_into(ctx, F64, cur, n, ld, f, ld_f, h, DIRICHLET0, r, ld_r, ctx->norms_dev, s))) return st;
    if ((st = read_norms(nr))) return st;
    bool r_fresh = true;  // r holds the residual of cur
    int backoff = 0, skip = 0;
    const double r0 = measure(nr);
    for (;;) {
        const double m = measure(nr);
        if (!std::isfinite(nr[0]) || !std::isfinite(nr[1])) { result = fail(PX_ENONFINITE, "non-finite residual"); break; }
        if (m <= target) break;
        if (m > 1e8 * std::max(r0, fref)) { result = fail(PX_EDIVERGED, "residual grew from %g to %g", r0, m); break; }
        if (S.base.sweeps >= o->max_sweeps) { result = fail(PX_ENOTCONV, "max_sweeps reached (rel res %g)", m / fref); break; }
        const int todo = (int)std::min<int64_t>(o->smooth_sweeps, o->max_sweeps - S.base.sweeps);
        if (correct && skip == 0) {
            if (!r_fresh &&
                (st = residual_into(ctx, F64, cur, n, ld, f, ld_f, h, DIRICHLET0, r, ld_r, ctx->norms_dev, s)))
                return st;
            PX_HIP(copy_grid_launch(F64, cur, save, n, ld, s), "copy kernel launch");
            const double rms = std::sqrt(nr[1] / ((double)n * (double)n));
            const void *d = r;
            int ddt = F64, ld_d = ld_r;
            if (o->use_net) {
                PX_HIP(net_infer(net, r, ld_r, n, 1.0 / rms, y, ld_y, s), "network forward launch");
                d = y;
                ddt = F32;
                ld_d = ld_y;
            }
            PX_HIP(correction_launch(ddt, d, ld_d, r, ld_r, static_cast<double *>(cur), n, ld, c, o->use_net, part,
                                     dots, nullptr, s),
                   "correction step launch");
            if ((st = smooth(todo, false))) return st;
            if ((st = residual_into(ctx, F64, cur, n, ld, f, ld_f, h, DIRICHLET0, r, ld_r, ctx->norms_dev, s)))
                return st;
            double nn[2];
            if ((st = read_norms(nn))) return st;
            const bool finite = std::isfinite(nn[0]) && std::isfinite(nn[1]);
            const bool better = finite && nn[1] < nr[1];
            if (better || (finite && o->judge != 2)) {
                S.corrections += 1;
                S.base.sweeps += todo;
                S.base.outer_steps += 1;
                nr[0] = nn[0];
                nr[1] = nn[1];
                r_fresh = true;
                if (better || o->judge == 0) {
                    backoff = 0;
                } else {
                    backoff = backoff ? std::min(2 * backoff, 64) : 1;
                    skip = backoff;
                }
            } else {
                // a broken network (non-finite) or, with judge 2, a step that raised the
                // residual: undo it
                PX_HIP(copy_grid_launch(F64, save, cur, n, ld, s), "copy kernel launch");
                S.rejected += 1;
                // the undone step's smoothing sweeps were run all the same: they count
                // against the budget and in the sweep total
                S.base.sweeps += todo;
                S.discarded_sweeps += todo;
                r_fresh = false;
                if (!finite) {
                    S.fell_back = 1;
                    correct = false;
                } else {
                    backoff = backoff ? std::min(2 * backoff, 64) : 1;
                    skip = backoff;
                }
            }
        } else {
            if ((st = smooth(todo, true))) return st;
            S.base.sweeps += todo;
            S.base.outer_steps += 1;
            r_fresh = false;
            if (skip > 0) skip -= 1;
            if ((st = read_norms(nr))) return st;
        }
    }
    if (cur != phi) PX_HIP(copy_grid_launch(F64, cur, phi, n, ld, s), "copy kernel launch");
    PX_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    S.base.res_max = nr[0];
    S.base.res_l2 = std::sqrt(nr[1]);
    S.base.rel_res_max = fn[0] > 0 ? nr[0] / fn[0] : nr[0];
    S.base.rel_res_l2 = fn[1] > 0 ? std::sqrt(nr[1] / fn[1]) : S.base.res_l2;
    S.base.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = S;
    return result;
}

}  // extern "C"
