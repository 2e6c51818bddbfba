// relax.hip -- host side of the fused relaxation: tile geometry, alignment
// checks and the choice of kernel instance (the kernel is in relax_kernel.h).
#include "relax_kernel.h"

namespace px {
using namespace relax_detail;
namespace {

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace

int relax_default_rows(int dtype, int n, int sweeps)
{
    // Measured on MI355X at 4096^2 (edge tiles launched first): FP64 favours tall bands at
    // 1-2 sweeps (fewer halo rows; waves stream long enough to hide latency), about 38 rows
    // at 3-6 sweeps and about 30 at 7-8, where the recomputed halo rows (about 2*sweeps
    // per band) weigh against the waves in flight; FP32 (256-column waves) about 20 rows
    // up to 7 sweeps.  With sweeps + 1 a multiple of 3 the interior loop runs in blocks of
    // sweeps + 1 steps, so the band height is chosen with rows + 2*sweeps a multiple of
    // sweeps + 1.
    int rows;
    if (dtype == F64)
        rows = sweeps <= 2 ? 48 : (sweeps <= 6 ? 38 : 32);
    else
        rows = sweeps <= 7 ? 20 : 32;
    // small grids are latency-bound: keep at least about 16 bands so more waves run at once
    rows = std::min(rows, std::max(8, (n + 2) / 16));
    if ((sweeps + 1) % 3 == 0) {
        const int u = sweeps + 1;
        rows -= (rows + 2 * sweeps) % u;  // largest such height not above the heuristic
        if (rows < 8) rows += u;
    }
    return rows;
}

int relax_num_waves(int dtype, int n, int sweeps, int resmode, int rows)
{
    const int NL = sweeps + (resmode == RES_FINAL ? 1 : 0);
    return make_geometry(vec_of(dtype), n, NL, rows).ntiles;
}

// Edge-first launch order (see launch_tile): the interior tiles, by the predicate
// relax_one_tile uses, form the rectangle [txl, txr) x [tyt, tyb).
static void set_launch_order(KArgs &ka, const Geometry &g, int V, int n, int NL, int nblocks)
{
    int txl = -1, txr = -1, tyt = -1, tyb = -1;
    for (int tx = 0; tx < g.tiles_x; ++tx) {
        const int c0 = g.col_origin + tx * g.stride - g.halo;
        if (c0 >= 1 && c0 + WAVE * V - (NL == 1 ? 0 : 1) <= n) {  // the predicate of relax_one_tile
            if (txl < 0) txl = tx;
            txr = tx + 1;
        }
    }
    for (int ty = 0; ty < g.tiles_y; ++ty) {
        const int y0 = ty * g.rows, y1 = std::min(y0 + g.rows, n + 2);
        if (y0 - NL >= 1 && y1 + NL - 1 <= n) {
            if (tyt < 0) tyt = ty;
            tyb = ty + 1;
        }
    }
    ka.edge_first = 0;
    ka.txl = ka.txr = ka.tyt = ka.tyb = ka.lead_blocks = 0;
    if (txl < 0 || tyt < 0) return;  // no interior tile: plain order
    const int nedge = g.ntiles - (txr - txl) * (tyb - tyt);
    ka.edge_first = 1;
    ka.txl = txl;
    ka.txr = txr;
    ka.tyt = tyt;
    ka.tyb = tyb;
    ka.lead_blocks = std::min(nblocks, ((nedge + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK + 7) / 8 * 8);
}

hipError_t relax_launch(int dtype, const RelaxLaunch &a, hipStream_t s)
{
    const int V = vec_of(dtype);
    const int NL = a.sweeps + (a.resmode == RES_FINAL ? 1 : 0);
    const Geometry g = make_geometry(V, a.n, NL, a.rows);
    const size_t es = (size_t)elem_size(dtype);
    KArgs ka;
    ka.in = a.in;
    ka.out = a.out;
    ka.f = a.f;
    ka.n = a.n;
    ka.ld = a.ld;
    ka.ld_f = a.ld_f;
    ka.bc = a.bc;
    ka.c = a.c;
    ka.w = a.w;
    ka.lam = a.lam;
    ka.halo = g.halo;
    ka.col_origin = g.col_origin;
    ka.stride = g.stride;
    ka.tiles_x = g.tiles_x;
    ka.rows = g.rows;
    ka.ntiles = g.ntiles;
    // vector loads/stores need every row start aligned to V elements
    const bool vec = aligned(a.in, V * es) && aligned(a.out, V * es) && a.ld % V == 0 &&
                     aligned(a.f, V * es) && a.ld_f % V == 0;
    // stream the output past the caches when phi, phi' and f together exceed the
    // 256 MB Infinity Cache
    const size_t ws = (2 * (size_t)(a.n + 2) * (size_t)a.ld + (size_t)a.n * (size_t)a.ld_f) * es;
    ka.nt_store = ws > ((size_t)256 << 20) ? 1 : 0;
    ka.pmax = a.part.max_bits;
    ka.psum = a.part.sum;
    LaunchFn fn = nullptr;
    switch (dtype) {
    case F64: fn = pick_f64(a.sweeps, a.resmode, vec); break;
    case F32: fn = pick_f32(a.sweeps, a.resmode, vec); break;
    case BF16: fn = pick_bf16(a.sweeps, a.resmode, vec); break;
    }
    if (!fn) return hipErrorInvalidValue;
    const int nblocks = (g.ntiles + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
    set_launch_order(ka, g, V, a.n, NL, nblocks);
    fn(ka, nblocks, s);
    return hipGetLastError();
}

}  // namespace px
