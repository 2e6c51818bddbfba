// relax_kernel.h -- fused, temporally blocked damped-Jacobi relaxation for gfx950.
//
// One kernel launch performs K sweeps (Section IV, Eq. 3 in the OL form
// phi' = (phi + w s) - lambda f with s the 5-point stencil of Eq. 1) and,
// on request, the max-norm of the residual (the OL norm expression), reading
// phi and f from HBM once and writing phi' once.
//
// Work decomposition ("2.5D" streaming, one wavefront = one tile):
//   * a wave owns 64*V consecutive columns (V elements per lane, 16 bytes for
//     FP64, 8 bytes for FP32/BF16 ... see VecOf) and a band of `rows` rows;
//   * it streams down its band one input row per step; level t (t = 1..K) of
//     the time pipeline is computed one row behind level t-1, from a 3-row
//     register window of level t-1, so all K sweeps happen in registers;
//   * east/west neighbours come from the adjacent lane with a cross-lane
//     shift, so no LDS and no barriers are needed -- waves are independent;
//   * the wave recomputes a halo of NL columns on each side and NL rows above
//     and below its band (overlapped tiling), so a tile's output depends only
//     on what the tile itself loaded.  Output columns per wave: `stride`.  (One
//     level: no column halo -- aligned strips, single-element neighbour loads.)
//   * edge tiles are launched first, then the interior in XCD-contiguous runs;
//     odd bands stream upwards, so neighbouring bands share halo rows via L2.
// Boundary: DIRICHLET0 replaces the neighbour across the boundary face by
// -(centre) at every level (odd reflection applied on the fly); GHOST_FIXED
// keeps ghost cells as fixed points of every level.
// Results are bit-identical to one sweep at a time: every level rounds to the
// storage type exactly as a store would, and the arithmetic order is fixed:
// s = ((((N - 4C) + W) + E) + S), phi' = (C + w s) - lambda f, r = f - c s.
//
// Partial norms are written per wave (max|r| as bit pattern, sum r^2 in a
// fixed lane/row order) and reduced in fixed order by reduce_partials().
#pragma once
#include "px_internal.h"

#include <algorithm>

namespace px {
namespace relax_detail {

constexpr int WAVE = 64;
constexpr int WAVES_PER_BLOCK = 4;
#ifndef PX_PREFETCH
#define PX_PREFETCH 2
#endif
constexpr int PREFETCH = PX_PREFETCH;  // input rows in flight ahead of the row being consumed

template <typename T> struct VecOf;
template <> struct VecOf<double> { static constexpr int V = 2; };
template <> struct VecOf<float> { static constexpr int V = 4; };
template <> struct VecOf<bf16> { static constexpr int V = 4; };

inline int vec_of(int dtype) { return dtype == F64 ? 2 : 4; }

struct Geometry {
    int halo, col_origin, stride, tiles_x, tiles_y, rows, ntiles;
};

// Column partition: a wave loads 64*V columns starting `halo` columns left of its
// output columns [col_origin + tx*stride, ... + stride).  halo >= NL (the columns
// each level invalidates at the wave's edges), rounded up to V so that loads and
// the output partition are both V-aligned.
inline Geometry make_geometry(int V, int n, int NL, int rows)
{
    Geometry g;
    // one pipeline level: no overlap -- waves own disjoint, 64 V-column strips that start on
    // 64 V-element boundaries, and the two columns beyond a strip come from single-element
    // loads (run_tile); deeper pipelines recompute a halo of NL columns, rounded to V
    g.halo = NL == 1 ? 0 : (NL + V - 1) / V * V;
    g.col_origin = 0;
    g.stride = WAVE * V - 2 * g.halo;
    g.tiles_x = (n + 2 + g.stride - 1) / g.stride;
    g.rows = rows;
    g.tiles_y = (n + 2 + rows - 1) / rows;
    g.ntiles = g.tiles_x * g.tiles_y;
    return g;
}

struct KArgs {
    const void *in;
    void *out;
    const void *f;
    int n, ld, ld_f, bc;
    double c, w, lam;
    int halo, col_origin, stride, tiles_x, rows, ntiles;
    int nt_store;  // non-temporal row stores (working set larger than the Infinity Cache)
    // edge-first launch order (0 = plain XCD-contiguous order): interior tiles are those
    // with txl <= tx < txr and tyt <= ty < tyb; the first lead_blocks blocks (a multiple
    // of 8) take the edge tiles
    int edge_first, txl, txr, tyt, tyb, lead_blocks;
    unsigned long long *pmax;
    double *psum;
};

// --- cross-lane shifts through DPP (a VALU operand modifier, no LDS traffic):
// wave_shr:1 gives lane l the value of lane l-1, wave_shl:1 that of lane l+1.
// Lanes at the ends of the wave receive 0; their columns are halo columns whose
// values are never used for an output.
constexpr int DPP_WAVE_SHR1 = 0x138;
constexpr int DPP_WAVE_SHL1 = 0x130;

// bound_ctrl: a lane without a source lane is written 0 (no "old" value to set up).
template <int CTRL>
__device__ __forceinline__ float dpp_shift(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <typename A> __device__ __forceinline__ A lane_from_left(A x) { return dpp_shift<DPP_WAVE_SHR1>(x); }
template <typename A> __device__ __forceinline__ A lane_from_right(A x) { return dpp_shift<DPP_WAVE_SHL1>(x); }

// --- memory access through buffer instructions.  A descriptor covers one row
// (wave-uniform, built with scalar instructions); the hardware returns 0 for
// loads and drops stores whose byte offset lies outside it, so a row outside the
// array gets a zero-sized descriptor and a masked lane gets the offset OOB.  No
// branches around loads: rows prefetched ahead stay in flight.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int RSRC_WORD3 = 0x00020000;  // raw (untyped) buffer, gfx9-family data format
constexpr int OOB = (int)0x80000000u;    // beyond every row descriptor (rows < 2 GiB)
// cache policy of a store: non-temporal (streamed past the caches).  Worth it when the
// grids of a launch do not fit the 256 MB Infinity Cache: each new row would otherwise
// push out input rows that other waves are about to read.
constexpr int CPOL_NT = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *base, int row, int nrows,
                                                           int row_bytes)
{
    const bool ok = row >= 0 && row < nrows;
    const char *p = static_cast<const char *>(base) + (size_t)(ok ? row : 0) * (size_t)row_bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, ok ? row_bytes : 0,
                                             RSRC_WORD3);
}

// A row stream: the address of row `row` of an array, moved one row per step by an add
// instead of a multiply per row.  The descriptor of a row outside [0, nrows) is zero-sized,
// as with row_rsrc, so its address is never dereferenced.
struct RowStream {
    const char *ptr;
    int row;
};
__device__ __forceinline__ RowStream row_stream(const void *base, int row, int row_bytes)
{
    return RowStream{static_cast<const char *>(base) + (long long)row * row_bytes, row};
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t stream_rsrc(const RowStream &s, int nrows, int row_bytes)
{
    const bool ok = (unsigned)s.row < (unsigned)nrows;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(s.ptr), (short)0, ok ? row_bytes : 0,
                                             RSRC_WORD3);
}
// The same with a zero-sized descriptor also when `need` is false (a prefetch of a row the
// tile does not use: the load returns zeros without touching memory).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t stream_rsrc_if(const RowStream &s, int nrows, int row_bytes,
                                                                bool need)
{
    const bool ok = need && (unsigned)s.row < (unsigned)nrows;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(s.ptr), (short)0, ok ? row_bytes : 0,
                                             RSRC_WORD3);
}
template <int D> __device__ __forceinline__ void step_stream(RowStream &s, int row_bytes)
{
    s.ptr += D > 0 ? (long long)row_bytes : -(long long)row_bytes;
    s.row += D;
}

// Raw load / store of V consecutive elements, as one vector access (VEC) or V
// scalar accesses.  Raw<T,V,VEC> holds the loaded bits until they are consumed.
template <typename T, int V, bool VEC> struct Io;

template <int V> struct Io<double, V, true> {
    static_assert(V == 2, "FP64 vector access is 16 bytes");
    using A = double;
    struct Raw { u32x4 u; };
    __device__ static Raw load(__amdgpu_buffer_rsrc_t r, int col0)
    {
        return Raw{__builtin_amdgcn_raw_buffer_load_b128(r, col0 * 8, 0, 0)};
    }
    __device__ static Raw load_cols(__amdgpu_buffer_rsrc_t r, const int (&col)[V])
    {
        const u32x2 a = __builtin_amdgcn_raw_buffer_load_b64(r, col[0] * 8, 0, 0);
        const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(r, col[1] * 8, 0, 0);
        u32x4 u;
        u.x = a.x;
        u.y = a.y;
        u.z = b.x;
        u.w = b.y;
        return Raw{u};
    }
    __device__ static void unpack(const Raw &x, A (&d)[V])
    {
        d[0] = __hiloint2double((int)x.u.y, (int)x.u.x);
        d[1] = __hiloint2double((int)x.u.w, (int)x.u.z);
    }
    __device__ static void store(__amdgpu_buffer_rsrc_t r, int off_elems, const A (&d)[V], bool nt)
    {
        u32x4 u;
        u.x = (unsigned)__double2loint(d[0]);
        u.y = (unsigned)__double2hiint(d[0]);
        u.z = (unsigned)__double2loint(d[1]);
        u.w = (unsigned)__double2hiint(d[1]);
        const int off = off_elems == OOB ? OOB : off_elems * 8;
        if (nt)
            __builtin_amdgcn_raw_buffer_store_b128(u, r, off, 0, CPOL_NT);
        else
            __builtin_amdgcn_raw_buffer_store_b128(u, r, off, 0, 0);
    }
};
template <int V> struct Io<double, V, false> {
    using A = double;
    struct Raw { u32x2 u[V]; };
    __device__ static Raw load(__amdgpu_buffer_rsrc_t r, int col0)
    {
        Raw x;
#pragma unroll
        for (int v = 0; v < V; ++v) x.u[v] = __builtin_amdgcn_raw_buffer_load_b64(r, (col0 + v) * 8, 0, 0);
        return x;
    }
    __device__ static Raw load_cols(__amdgpu_buffer_rsrc_t r, const int (&col)[V])
    {
        Raw x;
#pragma unroll
        for (int v = 0; v < V; ++v) x.u[v] = __builtin_amdgcn_raw_buffer_load_b64(r, col[v] * 8, 0, 0);
        return x;
    }
    __device__ static void unpack(const Raw &x, A (&d)[V])
    {
#pragma unroll
        for (int v = 0; v < V; ++v) d[v] = __hiloint2double((int)x.u[v].y, (int)x.u[v].x);
    }
};
template <int V> struct Io<float, V, true> {
    static_assert(V == 4, "FP32 vector access is 16 bytes");
    using A = float;
    struct Raw { u32x4 u; };
    __device__ static Raw load(__amdgpu_buffer_rsrc_t r, int col0)
    {
        return Raw{__builtin_amdgcn_raw_buffer_load_b128(r, col0 * 4, 0, 0)};
    }
    __device__ static Raw load_cols(__amdgpu_buffer_rsrc_t r, const int (&col)[V])
    {
        u32x4 u;
        u.x = __builtin_amdgcn_raw_buffer_load_b32(r, col[0] * 4, 0, 0);
        u.y = __builtin_amdgcn_raw_buffer_load_b32(r, col[1] * 4, 0, 0);
        u.z = __builtin_amdgcn_raw_buffer_load_b32(r, col[2] * 4, 0, 0);
        u.w = __builtin_amdgcn_raw_buffer_load_b32(r, col[3] * 4, 0, 0);
        return Raw{u};
    }
    __device__ static void unpack(const Raw &x, A (&d)[V])
    {
        d[0] = __uint_as_float(x.u.x);
        d[1] = __uint_as_float(x.u.y);
        d[2] = __uint_as_float(x.u.z);
        d[3] = __uint_as_float(x.u.w);
    }
    __device__ static void store(__amdgpu_buffer_rsrc_t r, int off_elems, const A (&d)[V], bool nt)
    {
        u32x4 u;
        u.x = __float_as_uint(d[0]);
        u.y = __float_as_uint(d[1]);
        u.z = __float_as_uint(d[2]);
        u.w = __float_as_uint(d[3]);
        const int off = off_elems == OOB ? OOB : off_elems * 4;
        if (nt)
            __builtin_amdgcn_raw_buffer_store_b128(u, r, off, 0, CPOL_NT);
        else
            __builtin_amdgcn_raw_buffer_store_b128(u, r, off, 0, 0);
    }
};
template <int V> struct Io<float, V, false> {
    using A = float;
    struct Raw { unsigned u[V]; };
    __device__ static Raw load(__amdgpu_buffer_rsrc_t r, int col0)
    {
        Raw x;
#pragma unroll
        for (int v = 0; v < V; ++v) x.u[v] = __builtin_amdgcn_raw_buffer_load_b32(r, (col0 + v) * 4, 0, 0);
        return x;
    }
    __device__ static Raw load_cols(__amdgpu_buffer_rsrc_t r, const int (&col)[V])
    {
        Raw x;
#pragma unroll
        for (int v = 0; v < V; ++v) x.u[v] = __builtin_amdgcn_raw_buffer_load_b32(r, col[v] * 4, 0, 0);
        return x;
    }
    __device__ static void unpack(const Raw &x, A (&d)[V])
    {
#pragma unroll
        for (int v = 0; v < V; ++v) d[v] = __uint_as_float(x.u[v]);
    }
};
template <int V> struct Io<bf16, V, true> {
    static_assert(V == 4, "BF16 vector access is 8 bytes");
    using A = float;
    struct Raw { u32x2 u; };
    __device__ static Raw load(__amdgpu_buffer_rsrc_t r, int col0)
    {
        return Raw{__builtin_amdgcn_raw_buffer_load_b64(r, col0 * 2, 0, 0)};
    }
    __device__ static Raw load_cols(__amdgpu_buffer_rsrc_t r, const int (&col)[V])
    {
        unsigned e[V];
#pragma unroll
        for (int v = 0; v < V; ++v) e[v] = (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, col[v] * 2, 0, 0);
        u32x2 u;
        u.x = e[0] | (e[1] << 16);
        u.y = e[2] | (e[3] << 16);
        return Raw{u};
    }
    __device__ static void unpack(const Raw &x, A (&d)[V])
    {
        d[0] = __uint_as_float(x.u.x << 16);
        d[1] = __uint_as_float(x.u.x & 0xffff0000u);
        d[2] = __uint_as_float(x.u.y << 16);
        d[3] = __uint_as_float(x.u.y & 0xffff0000u);
    }
    __device__ static void store(__amdgpu_buffer_rsrc_t r, int off_elems, const A (&d)[V], bool nt)
    {
        u32x2 u;
        u.x = (unsigned)f32_to_bf16_rne(d[0]) | ((unsigned)f32_to_bf16_rne(d[1]) << 16);
        u.y = (unsigned)f32_to_bf16_rne(d[2]) | ((unsigned)f32_to_bf16_rne(d[3]) << 16);
        const int off = off_elems == OOB ? OOB : off_elems * 2;
        if (nt)
            __builtin_amdgcn_raw_buffer_store_b64(u, r, off, 0, CPOL_NT);
        else
            __builtin_amdgcn_raw_buffer_store_b64(u, r, off, 0, 0);
    }
};
template <int V> struct Io<bf16, V, false> {
    using A = float;
    struct Raw { unsigned short u[V]; };
    __device__ static Raw load(__amdgpu_buffer_rsrc_t r, int col0)
    {
        Raw x;
#pragma unroll
        for (int v = 0; v < V; ++v) x.u[v] = __builtin_amdgcn_raw_buffer_load_b16(r, (col0 + v) * 2, 0, 0);
        return x;
    }
    __device__ static Raw load_cols(__amdgpu_buffer_rsrc_t r, const int (&col)[V])
    {
        Raw x;
#pragma unroll
        for (int v = 0; v < V; ++v) x.u[v] = __builtin_amdgcn_raw_buffer_load_b16(r, col[v] * 2, 0, 0);
        return x;
    }
    __device__ static void unpack(const Raw &x, A (&d)[V])
    {
#pragma unroll
        for (int v = 0; v < V; ++v) d[v] = __uint_as_float((unsigned)x.u[v] << 16);
    }
};

// Single-element load of column col (OOB: 0), as the arithmetic type.
template <typename T> struct Load1;
template <> struct Load1<double> {
    __device__ static double ld(__amdgpu_buffer_rsrc_t r, int col)
    {
        const u32x2 u = __builtin_amdgcn_raw_buffer_load_b64(r, col == OOB ? OOB : col * 8, 0, 0);
        return __hiloint2double((int)u.y, (int)u.x);
    }
};
template <> struct Load1<float> {
    __device__ static float ld(__amdgpu_buffer_rsrc_t r, int col)
    {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, col == OOB ? OOB : col * 4, 0, 0));
    }
};
template <> struct Load1<bf16> {
    __device__ static float ld(__amdgpu_buffer_rsrc_t r, int col)
    {
        return __uint_as_float((unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, col == OOB ? OOB : col * 2, 0, 0)
                               << 16);
    }
};

// Single-element masked store (edge tiles, ghost cells).
__device__ __forceinline__ void store1(__amdgpu_buffer_rsrc_t r, int col, bool ok, double x)
{
    u32x2 u;
    u.x = (unsigned)__double2loint(x);
    u.y = (unsigned)__double2hiint(x);
    __builtin_amdgcn_raw_buffer_store_b64(u, r, ok ? col * 8 : OOB, 0, 0);
}
__device__ __forceinline__ void store1_f(__amdgpu_buffer_rsrc_t r, int col, bool ok, float x)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, ok ? col * 4 : OOB, 0, 0);
}
__device__ __forceinline__ void store1_b(__amdgpu_buffer_rsrc_t r, int col, bool ok, float x)
{
    __builtin_amdgcn_raw_buffer_store_b16(f32_to_bf16_rne(x), r, ok ? col * 2 : OOB, 0, 0);
}
template <typename T> struct Store1;
template <> struct Store1<double> {
    __device__ static void st(__amdgpu_buffer_rsrc_t r, int c, bool ok, double x) { store1(r, c, ok, x); }
};
template <> struct Store1<float> {
    __device__ static void st(__amdgpu_buffer_rsrc_t r, int c, bool ok, float x) { store1_f(r, c, ok, x); }
};
template <> struct Store1<bf16> {
    __device__ static void st(__amdgpu_buffer_rsrc_t r, int c, bool ok, float x) { store1_b(r, c, ok, x); }
};

// Stores the elements of V consecutive columns col0.. that fall in [lo, hi),
// negated if asked.  Whole vectors when the tile is known to hold only whole
// vectors (`whole`, wave-uniform), element by element otherwise.
template <typename T, int V, bool VEC>
__device__ __forceinline__ void store_cols(__amdgpu_buffer_rsrc_t r, int col0, int lo, int hi,
                                           bool whole, const typename Elem<T>::A (&val)[V], bool negate,
                                           bool nt = false)
{
    using A = typename Elem<T>::A;
    A x[V];
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = negate ? -val[v] : val[v];
    if constexpr (VEC) {
        if (whole) {
            Io<T, V, true>::store(r, (col0 >= lo && col0 + V <= hi) ? col0 : OOB, x, nt);
            return;
        }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) Store1<T>::st(r, col0 + v, col0 + v >= lo && col0 + v < hi, x[v]);
}

// Periodic grids: row or column x of the ghosted index space (any x, ghosts and halo
// included) as the interior cell of the torus it stands for, in [1, n].
__device__ __forceinline__ int torus(int x, int n)
{
    int r = (x - 1) % n;
    if (r < 0) r += n;
    return r + 1;
}

// Geometry of one wave's tile (wave-uniform except mc).
struct Tile {
    int n, oc0, oc1, mc, y0, y1;
    bool whole;  // only whole vectors of interior columns to store
};

// The streaming loop of one tile.  EDGE = false is the interior-tile path: every cell
// the wave computes is an interior cell, so no boundary substitution, no ghost writes
// and no selects on the update -- the common case, taken when the tile's loaded
// columns and needed rows all lie in [1, n].
template <typename T, int V, int K, int RM, int PF, bool VEC, bool EDGE, bool PER = false>
__device__ __forceinline__ void run_tile(const KArgs &p, const Tile &tl, unsigned long long &rmax,
                                         double &rsum)
{
    using E = Elem<T>;
    using A = typename E::A;
    using IO = Io<T, V, VEC>;
    using Raw = typename IO::Raw;
    constexpr int NL = K + (RM == RES_FINAL ? 1 : 0);
    constexpr int RL = (RM == RES_FINAL) ? K + 1 : K;
    constexpr int FQ = RL + 1;
    constexpr int ES = (int)sizeof(T);
    // one level, no halo: the strip's outer neighbours come from single-element loads of
    // each row (lane 0 the column left of the strip, the last lane the one right of it), and
    // lane 0's f of its first column (which the one-column shift of f would take from the
    // strip to the left) from one more
    constexpr bool NH = (NL == 1);
    const int n = tl.n, oc0 = tl.oc0, oc1 = tl.oc1, mc = tl.mc, y0 = tl.y0, y1 = tl.y1;
    const int lane = threadIdx.x & (WAVE - 1);
    const int c0 = mc - lane * V;
    const bool whole = tl.whole;
    const bool dir = (p.bc == DIRICHLET0);
    // periodic grid (edge tiles only: an interior tile never reaches the ghost ring): rows
    // and columns of every load wrap onto the torus, and every cell is computed and
    // stored, the ghost ring and its corners included, so no boundary substitution
    constexpr bool per = EDGE && PER;  // a separate instance: no wrap tests in the others
    const int ecol = per ? (lane == 0 ? torus(c0 - 1, n) : (lane == WAVE - 1 ? torus(c0 + WAVE * V, n) : OOB))
                         : ((lane == 0) ? (c0 >= 1 ? c0 - 1 : OOB) : (lane == WAVE - 1 ? c0 + WAVE * V : OOB));
    // f is compact: f column j - 1 belongs to phi column j
    const int efcol = (VEC && lane == 0) ? (per ? torus(c0, n) - 1 : (c0 >= 1 ? c0 - 1 : OOB)) : OOB;
    const int rb = p.ld * ES, rbf = p.ld_f * ES;
    const A w = (A)p.w, cc = (A)p.c, lam = (A)p.lam;

    A win[NL][3][V];
    A fq[FQ][V];
#pragma unroll
    for (int t = 0; t < NL; ++t)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int v = 0; v < V; ++v) win[t][k][v] = 0;
#pragma unroll
    for (int j = 0; j < FQ; ++j)
#pragma unroll
        for (int v = 0; v < V; ++v) fq[j][v] = 0;

    // residual window of this wave: rows [ry0, ry1), columns [rc0, rc1), interior only
    const int ry0 = max(y0, 1), ry1 = min(y1, n + 1);
    const int rc0 = max(oc0, 1), rc1 = min(oc1, n + 1);
    // columns of f loaded by this lane: its own aligned columns (VEC, shifted by one
    // lane afterwards) or exactly the columns its cells need
    const int fc = VEC ? mc : mc - 1;
    // the loads of one row of phi and f (and the strip's outer neighbours), wrapped on a torus
    int pcol[V], fcol[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        pcol[v] = per ? torus(mc + v, n) : 0;
        fcol[v] = per ? torus(fc + v + 1, n) - 1 : 0;
    }
    auto load_phi = [&](int row) -> Raw {
        if constexpr (per) return IO::load_cols(row_rsrc(p.in, torus(row, n), n + 2, rb), pcol);
        return IO::load(row_rsrc(p.in, row, n + 2, rb), mc);
    };
    auto load_f = [&](int row) -> Raw {  // f of phi row `row`
        if constexpr (per) return IO::load_cols(row_rsrc(p.f, torus(row, n) - 1, n, rbf), fcol);
        return IO::load(row_rsrc(p.f, row - 1, n, rbf), fc);
    };
    auto load1_phi = [&](int row) -> A {
        return Load1<T>::ld(row_rsrc(p.in, per ? torus(row, n) : row, n + 2, rb), ecol);
    };
    auto load1_f = [&](int row) -> A {
        return Load1<T>::ld(row_rsrc(p.f, (per ? torus(row, n) : row) - 1, n, rbf), efcol);
    };

    // Rows are prefetched PF ahead into a ring of raw registers; the loop is
    // unrolled PF times so the ring rotates by renaming, never by moves that would
    // wait on loads in flight.
    // (the step count is rounded up to a multiple of PF: the extra steps compute
    // rows past the band and store nothing, and the loop keeps a single latch)
    const int sb = y0 - NL, se = sb + (y1 - y0 + 2 * NL + PF - 1) / PF * PF;
    Raw pf[PF], pff[PF];
    A pe[NH ? PF : 1], pfe[NH ? PF : 1];  // single-element loads of the rows in flight
    A ex1 = 0, ex2 = 0;                    // single elements of rows s - 1, s
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        pf[q] = load_phi(sb + q);
        pff[q] = load_f(sb + q);
        if constexpr (NH) {
            pe[q] = load1_phi(sb + q);
            pfe[q] = load1_f(sb + q);
        }
    }
    for (int s0 = sb; s0 < se; s0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int s = s0 + q;
            // ---- level 0: row s of phi and of f from the ring, then refill the slot
#pragma unroll
            for (int v = 0; v < V; ++v) {
                win[0][0][v] = win[0][1][v];
                win[0][1][v] = win[0][2][v];
            }
            IO::unpack(pf[q], win[0][2]);
            if constexpr (NH) {
                ex1 = ex2;
                ex2 = pe[q];
            }
#pragma unroll
            for (int j = FQ - 1; j > 0; --j)
#pragma unroll
                for (int v = 0; v < V; ++v) fq[j][v] = fq[j - 1][v];
            {
                A fo[V];
                IO::unpack(pff[q], fo);
                if constexpr (VEC) {
                    const A sh = lane_from_left(fo[V - 1]);
                    fq[0][0] = (NH && lane == 0) ? pfe[NH ? q : 0] : sh;
#pragma unroll
                    for (int v = 1; v < V; ++v) fq[0][v] = fo[v - 1];
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) fq[0][v] = fo[v];
                }
            }
            pf[q] = load_phi(s + PF);
            pff[q] = load_f(s + PF);
            if constexpr (NH) {
                pe[q] = load1_phi(s + PF);
                pfe[q] = load1_f(s + PF);
            }

            // ---- levels 1..NL, level t at row s - t
#pragma unroll
            for (int t = 1; t <= NL; ++t) {
                if (s < y0 - NL + 2 * t) break;  // rows this level does not need yet
                const int r = s - t;
                A left = lane_from_left(win[t - 1][1][V - 1]);
                A right = lane_from_right(win[t - 1][1][0]);
                if constexpr (NH) {
                    left = lane == 0 ? ex1 : left;
                    right = lane == WAVE - 1 ? ex1 : right;
                }
                A st[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const A C = win[t - 1][1][v];
                    A N = win[t - 1][0][v];
                    A S = win[t - 1][2][v];
                    A Wn = (v == 0) ? left : win[t - 1][1][v - 1];
                    A En = (v == V - 1) ? right : win[t - 1][1][v + 1];
                    if (EDGE && dir) {
                        const int col = mc + v;
                        if (r == 1) N = -C;
                        if (r == n) S = -C;
                        if (col == 1) Wn = -C;
                        if (col == n) En = -C;
                    }
                    st[v] = ((sub4(N, C) + Wn) + En) + S;
                }
                if (t <= K) {
                    A nv[V];
                    const bool row_in = (r >= 1 && r <= n);
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const int col = mc + v;
                        const A C = win[t - 1][1][v];
                        const A u = E::round((C + w * st[v]) - lam * fq[t][v]);
                        const bool inter = row_in && col >= 1 && col <= n;
                        nv[v] = EDGE ? ((inter || per) ? u : (dir ? (A)0 : C)) : u;
                    }
                    if (t < NL) {
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            win[t][0][v] = win[t][1][v];
                            win[t][1][v] = win[t][2][v];
                            win[t][2][v] = nv[v];
                        }
                    }
                    if (t == K && r >= y0 && r < y1) {
                        if constexpr (!EDGE) {
                            // interior tile: interior rows and columns only, whole vectors
                            store_cols<T, V, VEC>(row_rsrc(p.out, r, n + 2, rb), mc, oc0, oc1, true, nv,
                                                  false, p.nt_store != 0);
                        } else if (dir) {
                            if (row_in) {
                                const auto ro = row_rsrc(p.out, r, n + 2, rb);
                                store_cols<T, V, VEC>(ro, mc, rc0, rc1, whole, nv, false);
                                if (!whole) {
                                    // edge ghosts of this row: -(column 1), -(column n)
#pragma unroll
                                    for (int v = 0; v < V; ++v) {
                                        const int col = mc + v;
                                        const bool mine = col >= rc0 && col < rc1;
                                        Store1<T>::st(ro, 0, mine && col == 1, -nv[v]);
                                        Store1<T>::st(ro, n + 1, mine && col == n, -nv[v]);
                                    }
                                }
                                // ghost rows 0 and n+1 mirror rows 1 and n
                                if (r == 1)
                                    store_cols<T, V, VEC>(row_rsrc(p.out, 0, n + 2, rb), mc, rc0, rc1,
                                                          whole, nv, true);
                                if (r == n)
                                    store_cols<T, V, VEC>(row_rsrc(p.out, n + 1, n + 2, rb), mc, rc0,
                                                          rc1, whole, nv, true);
                            }
                        } else {
                            // fixed ghosts: the ghost ring keeps its values, corners untouched;
                            // torus: the ghost ring and its corners hold their wrapped cells
                            const bool skip_corners = (r == 0 || r == n + 1) && !per;
                            const int lo = max(oc0, skip_corners ? 1 : 0);
                            const int hi = min(oc1, skip_corners ? n + 1 : n + 2);
                            store_cols<T, V, VEC>(row_rsrc(p.out, r, n + 2, rb), mc, lo, hi,
                                                  whole && !skip_corners, nv, false);
                        }
                    }
                }
                if (RM != RES_NONE && t == RL && r >= ry0 && r < ry1) {
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const int col = mc + v;
                        const A rr = fq[t][v] - cc * st[v];
                        const double rd = (double)rr;
                        const unsigned long long bits =
                            (unsigned long long)__double_as_longlong(fabs(rd));
                        const bool mine = col >= rc0 && col < rc1;
                        rmax = (mine && bits > rmax) ? bits : rmax;
                        rsum += mine ? rd * rd : 0.0;
                    }
                }
            }
        }
    }

}

// Tiles of launches without norms whose K + 1 is a multiple of 3 (K = 2, 5, 8) -- interior
// tiles, and with EDGE the edge tiles of homogeneous-Dirichlet grids, which keep the ghost
// cells of every level at the odd reflection (below) and write the ghost layer: the step
// loop is unrolled U = K + 1 times, so the 3-row windows of every level (3 | U), the
// (K + 1)-row ring of lambda f (U rows) and a 3-deep ring of prefetched rows all rotate by
// renaming: the row of step v of a level lives in slot v mod 3, lambda f of the phi row
// of step v in slot v mod U.  The product lambda f is formed once per row when the row
// arrives and reused by all K levels: the same rounded product each level would form, so
// the results are those of run_tile bit for bit.  Level t starts 2t steps after the first
// row; the first blocks of U steps (the pipeline filling up) test which levels are active,
// the rest run every level unconditionally.  The step count is rounded up to a multiple of
// U (the extra steps compute rows past the band and store nothing).
//
// UP streams the band from its bottom row upwards.  The arithmetic is unchanged -- N is
// still the row above and S the row below, summed in the same order -- only the step that
// delivers each row differs.  Bands alternate direction, so two neighbouring bands read the
// 2K rows they share at the same end of their lives (both first or both last) while they
// run side by side, and the second read of a shared row tends to hit the L2.
template <typename T, int V, int K, bool VEC, bool FILLING, bool UP, bool EDGE, int COLS = 0,
          bool ROWFIX = false>
__device__ __forceinline__ void renamed_block(const KArgs &p, const Tile &tl, int s0, int base,
                                              typename Elem<T>::A (&win)[K][3][V],
                                              typename Elem<T>::A (&lf)[K + 1][V],
                                              typename Io<T, V, VEC>::Raw (&pf)[3],
                                              typename Io<T, V, VEC>::Raw (&pff)[3],
                                              RowStream &sin, RowStream &sfr, RowStream &sout)
{
    using E = Elem<T>;
    using A = typename E::A;
    using IO = Io<T, V, VEC>;
    constexpr int U = K + 1;
    constexpr int PR = 3;
    constexpr int ES = (int)sizeof(T);
    constexpr int M3 = 3 * U;  // keeps the slot arithmetic non-negative
    constexpr int D = UP ? -1 : 1;  // row step of the stream
    const int n = tl.n, oc0 = tl.oc0, oc1 = tl.oc1, mc = tl.mc, y0 = tl.y0, y1 = tl.y1;
    const int rb = p.ld * ES, rbf = p.ld_f * ES;
    const A w = (A)p.w, lam = (A)p.lam;
    const int fc = VEC ? mc : mc - 1;
    const int nsteps = y1 - y0 + 2 * K;  // steps whose input row the tile uses
    // Edge tiles (homogeneous Dirichlet) keep the ghost cells of every time level equal to
    // the odd reflection of their neighbours inside, as a refresh of the ghost layer
    // before each sweep would: after each level's row is formed, column 0 := -column 1 and
    // column n + 1 := -column n in the waves that hold them (COLS: 1 column 0, 2 column
    // n + 1 in the lane of column n, 3 both or column n + 1 starting a lane; column 0 is
    // element 0 of a lane since waves start on multiples of V), and the ghost rows 0 and
    // n + 1 := -rows 1 and n, whichever of each pair comes second in the stream being set
    // when it does (ROWFIX).  Every interior cell then reads the value the substitution
    // N = -C (or S, W, E) gives, with the interior arithmetic.  The column rule is one
    // select per level in the waves at the left or right edge, and the row rule runs only
    // while the pipeline fills (bands that reach a ghost row stream away from it), so the
    // code of the other blocks stays as straight as the interior tiles'.
    const bool rowtile = y0 - K <= 1 || y1 + K - 1 >= n;  // the band reaches a ghost row
    auto ghost_cols = [&](A(&a)[V]) {
        if constexpr (COLS == 1 || COLS == 3) a[0] = (mc == 0) ? -a[1] : a[0];
        if constexpr (COLS >= 2) {
#pragma unroll
            for (int v = 1; v < V; ++v) a[v] = (mc + v == n + 1) ? -a[v - 1] : a[v];
        }
        if constexpr (COLS == 3) {
            const A pl = lane_from_left(a[V - 1]);
            a[0] = (mc == n + 1) ? -pl : a[0];
        }
    };
#pragma unroll
    for (int q = 0; q < U; ++q) {
        const int s = s0 + q;       // step
        const int x = base + D * s;  // phi row arriving at this step
        IO::unpack(pf[q % PR], win[0][q % 3]);
        if constexpr (EDGE && COLS != 0) ghost_cols(win[0][q % 3]);  // the same rules for the input rows
        if constexpr (EDGE && ROWFIX) {
            if (rowtile) {  // side strips of the middle bands skip the row rule
                const int pq = (q + 2) % 3;  // slot of the previous step's row
                const bool second = x == (UP ? 0 : n + 1), first = x == (UP ? n : 1);
#pragma unroll
                for (int v = 0; v < V; ++v) win[0][q % 3][v] = second ? -win[0][pq][v] : win[0][q % 3][v];
#pragma unroll
                for (int v = 0; v < V; ++v) win[0][pq][v] = first ? -win[0][q % 3][v] : win[0][pq][v];
            }
        }
        {
            A fo[V], fv[V];
            IO::unpack(pff[q % PR], fo);
            if constexpr (VEC) {
                fv[0] = lane_from_left(fo[V - 1]);
#pragma unroll
                for (int v = 1; v < V; ++v) fv[v] = fo[v - 1];
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) fv[v] = fo[v];
            }
#pragma unroll
            for (int v = 0; v < V; ++v) lf[q][v] = lam * fv[v];
        }
        // rows x + D PR of phi and f (streams sin, sfr); level K stores row x - D K (sout)
        // (the last PR steps of the tile's rows need no further rows: their loads stay
        // off memory -- the steps past them, up to a multiple of U, form no stored row)
        const bool more = s + PR < nsteps;
        pf[q % PR] = IO::load(stream_rsrc_if(sin, n + 2, rb, more), mc);
        pff[q % PR] = IO::load(stream_rsrc_if(sfr, n, rbf, more), fc);
        step_stream<D>(sin, rb);
        step_stream<D>(sfr, rbf);
#pragma unroll
        for (int t = 1; t <= K; ++t) {
            if (FILLING && s < 2 * t) break;  // rows this level does not need yet
            const int r = x - D * t;          // row level t computes
            const int so = (q - t - 1 + M3) % 3, sc = (q - t + M3) % 3, sw = (q - t + 1 + M3) % 3;
            const int sn = UP ? sw : so, ss = UP ? so : sw;  // slots of rows r - 1 and r + 1
            const int sf = (q - t + U) % U;
            const A left = lane_from_left(win[t - 1][sc][V - 1]);
            const A right = lane_from_right(win[t - 1][sc][0]);
            A nv[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const A C = win[t - 1][sc][v];
                const A N = win[t - 1][sn][v];
                const A S = win[t - 1][ss][v];
                const A Wn = (v == 0) ? left : win[t - 1][sc][v - 1];
                const A En = (v == V - 1) ? right : win[t - 1][sc][v + 1];
                const A st = ((sub4(N, C) + Wn) + En) + S;
                nv[v] = E::round((C + w * st) - lf[sf][v]);
            }
            if constexpr (EDGE && COLS != 0) ghost_cols(nv);
            if (t < K) {
                if constexpr (EDGE && ROWFIX) {
                    if (rowtile) {
                        // the second ghost row of its pair takes the mirror of the row before
                        // it; the first is set once the row after it (its mirror) is formed
                        const bool second = r == (UP ? 0 : n + 1), first = r == (UP ? n : 1);
#pragma unroll
                        for (int v = 0; v < V; ++v) nv[v] = second ? -win[t][so][v] : nv[v];
#pragma unroll
                        for (int v = 0; v < V; ++v) win[t][so][v] = first ? -nv[v] : win[t][so][v];
                    }
                }
#pragma unroll
                for (int v = 0; v < V; ++v) win[t][sc][v] = nv[v];
            } else if (UP ? r >= y0 : r < y1) {  // the other bound holds once level K runs
                if constexpr (!EDGE) {
                    store_cols<T, V, VEC>(stream_rsrc(sout, n + 2, rb), mc, oc0, oc1, true, nv, false,
                                          p.nt_store != 0);
                } else if constexpr (!ROWFIX) {
                    // rows 2 .. n - 1 only: the row with its ghost columns
                    const int hi = min(oc1, n + 2);
                    store_cols<T, V, VEC>(stream_rsrc(sout, n + 2, rb), mc, oc0, hi, oc0 % V == 0 && hi % V == 0,
                                          nv, false, p.nt_store != 0);
                } else if (r >= 1 && r <= n) {
                    // the row with its ghost columns (which hold the mirrors of columns 1
                    // and n), and the ghost rows 0 and n + 1 as the mirrors of rows 1 and n
                    // (the four corners are left untouched)
                    const int rc0 = max(oc0, 1), rc1 = min(oc1, n + 1), hi = min(oc1, n + 2);
                    const bool nt = p.nt_store != 0;
                    // whole vectors when both ends of the stored range fall on vector bounds
                    store_cols<T, V, VEC>(stream_rsrc(sout, n + 2, rb), mc, oc0, hi, oc0 % V == 0 && hi % V == 0,
                                          nv, false, nt);
                    if (r == 1)
                        store_cols<T, V, VEC>(row_rsrc(p.out, 0, n + 2, rb), mc, rc0, rc1, tl.whole, nv, true, nt);
                    if (r == n)
                        store_cols<T, V, VEC>(row_rsrc(p.out, n + 1, n + 2, rb), mc, rc0, rc1, tl.whole, nv, true,
                                              nt);
                }
            }
        }
        step_stream<D>(sout, rb);
    }
}

template <typename T, int V, int K, bool VEC, bool UP, bool EDGE, int COLS = 0>
__device__ __forceinline__ void run_tile_renamed(const KArgs &p, const Tile &tl)
{
    using E = Elem<T>;
    using A = typename E::A;
    using IO = Io<T, V, VEC>;
    using Raw = typename IO::Raw;
    constexpr int U = K + 1;
    constexpr int PR = 3;
    static_assert(U % 3 == 0, "window slots must repeat within the unrolled steps");
    constexpr int ES = (int)sizeof(T);
    constexpr int D = UP ? -1 : 1;
    const int n = tl.n, mc = tl.mc, y0 = tl.y0, y1 = tl.y1;
    const int rb = p.ld * ES, rbf = p.ld_f * ES;

    A win[K][3][V];
    A lf[U][V];
#pragma unroll
    for (int t = 0; t < K; ++t)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int v = 0; v < V; ++v) win[t][k][v] = 0;
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
        for (int v = 0; v < V; ++v) lf[j][v] = 0;
    const int fc = VEC ? mc : mc - 1;
    const int base = UP ? y1 - 1 + K : y0 - K;  // first row of the stream
    const int steps = (y1 - y0 + 2 * K + U - 1) / U * U;
    Raw pf[PR], pff[PR];
#pragma unroll
    for (int q = 0; q < PR; ++q) {
        pf[q] = IO::load(row_rsrc(p.in, base + D * q, n + 2, rb), mc);
        pff[q] = IO::load(row_rsrc(p.f, base + D * q - 1, n, rbf), fc);
    }
    RowStream sin = row_stream(p.in, base + D * PR, rb), sfr = row_stream(p.f, base + D * PR - 1, rbf),
              sout = row_stream(p.out, base - D * K, rb);
    int s0 = 0;
    if constexpr (!EDGE) {
        for (; s0 < steps && s0 < 2 * K; s0 += U)
            renamed_block<T, V, K, VEC, true, UP, false>(p, tl, s0, base, win, lf, pf, pff, sin, sfr, sout);
        for (; s0 < steps; s0 += U)
            renamed_block<T, V, K, VEC, false, UP, false>(p, tl, s0, base, win, lf, pf, pff, sin, sfr, sout);
    } else {
        // Bands that reach a ghost row stream away from it (relax_one_tile), so every row
        // within K + 1 of it is formed in the first 2K + 2 steps: the two blocks that fill
        // the pipeline, which alone apply the ghost-row rule.
        for (; s0 < steps && s0 < 2 * K; s0 += U)
            renamed_block<T, V, K, VEC, true, UP, true, COLS, true>(p, tl, s0, base, win, lf, pf, pff, sin, sfr,
                                                                   sout);
        for (; s0 < steps; s0 += U)
            renamed_block<T, V, K, VEC, false, UP, true, COLS, false>(p, tl, s0, base, win, lf, pf, pff, sin, sfr,
                                                                     sout);
    }
}

// One wave tile of one problem: geometry, interior/edge dispatch, streaming loop.
template <typename T, int V, int K, int RM, int PF, bool VEC>
__device__ __forceinline__ void relax_one_tile(const KArgs &p, int tile, int lane, unsigned long long &rmax,
                                               double &rsum)
{
    constexpr int NL = K + (RM == RES_FINAL ? 1 : 0);  // pipeline levels
    const int n = p.n;
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int oc0 = p.col_origin + tx * p.stride;  // output columns [oc0, oc1)
    const int oc1 = min(oc0 + p.stride, n + 2);
    const int c0 = oc0 - p.halo;                   // first column held by the wave
    const int mc = c0 + lane * V;                  // first column held by this lane
    const int y0 = ty * p.rows, y1 = min(y0 + p.rows, n + 2);
    // tiles whose outputs avoid columns 0, 1, n, n+1 store whole vectors
    const bool whole = oc0 >= V && oc1 <= n;
    // interior tile: loaded columns and needed rows all inside [1, n] (with one level the
    // strip also reads the column right of it, which must not be the ghost column n + 1)
    const bool interior = c0 >= 1 && c0 + WAVE * V - (NL == 1 ? 0 : 1) <= n && y0 - NL >= 1 && y1 + NL - 1 <= n;
    const Tile tl{n, oc0, oc1, mc, y0, y1, whole};
    if constexpr (RM == RES_NONE && (K + 1) % 3 == 0) {
        const bool up = (ty & 1) != 0;
        if (interior) {
            if (up)
                run_tile_renamed<T, V, K, VEC, true, false>(p, tl);
            else
                run_tile_renamed<T, V, K, VEC, false, false>(p, tl);
            return;
        }
        // Dirichlet edge tiles: a band whose rows reach ghost row 0 streams down and one
        // that reaches ghost row n + 1 streams up (so the ghost-row rule is needed only while
        // the pipeline fills); a band reaching both takes the general path
        const bool top = y0 - K <= 1, bot = y1 + K - 1 >= n;
        if (p.bc == DIRICHLET0 && !(top && bot)) {
            const bool up = bot || (!top && (ty & 1) != 0);
            const bool hw = c0 <= 0, he = c0 + WAVE * V > n + 1;  // the wave holds column 0 / n + 1
            const int cm = ((hw && he) || (he && (n + 1) % V == 0)) ? 3 : (hw ? 1 : (he ? 2 : 0));
            switch (cm + (up ? 4 : 0)) {
            case 0: run_tile_renamed<T, V, K, VEC, false, true, 0>(p, tl); break;
            case 1: run_tile_renamed<T, V, K, VEC, false, true, 1>(p, tl); break;
            case 2: run_tile_renamed<T, V, K, VEC, false, true, 2>(p, tl); break;
            case 3: run_tile_renamed<T, V, K, VEC, false, true, 3>(p, tl); break;
            case 4: run_tile_renamed<T, V, K, VEC, true, true, 0>(p, tl); break;
            case 5: run_tile_renamed<T, V, K, VEC, true, true, 1>(p, tl); break;
            case 6: run_tile_renamed<T, V, K, VEC, true, true, 2>(p, tl); break;
            default: run_tile_renamed<T, V, K, VEC, true, true, 3>(p, tl); break;
            }
            return;
        }
    }
    if (interior)
        run_tile<T, V, K, RM, PF, VEC, false>(p, tl, rmax, rsum);
    else if (p.bc == PERIODIC)
        run_tile<T, V, K, RM, PF, VEC, true, true>(p, tl, rmax, rsum);
    else
        run_tile<T, V, K, RM, PF, VEC, true>(p, tl, rmax, rsum);
}

// Wave reduction of the partial norms in a fixed order (result in every lane).
__device__ __forceinline__ void wave_reduce_norms(unsigned long long &rmax, double &rsum, int lane)
{
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        const unsigned long long om = __shfl_xor(rmax, off, WAVE);
        const double os = __shfl_xor(rsum, off, WAVE);
        rmax = om > rmax ? om : rmax;
        // fixed pairing: the lower lane's value always comes first
        rsum = (lane & off) ? (os + rsum) : (rsum + os);
    }
}

// XCD-aware block order: block b runs on XCD b % 8; give each XCD a contiguous run
// of tiles so neighbouring tiles (shared halo rows/columns) share an L2.
__device__ __forceinline__ int xcd_block()
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int nb8 = nb & ~7;
    return (b < nb8) ? ((b & 7) * (nb8 >> 3) + (b >> 3)) : b;
}

// Launch order.  Edge tiles (boundary substitution and ghost writes: longer-lived than
// interior waves, by a factor up to 2.5 where they take run_tile) go first, spread over
// all XCDs, so that no slow wave starts near the end of the launch and stretches its
// tail; the interior tiles follow, each XCD taking a contiguous run.  Returns the tile
// index (ty * tiles_x + tx), or ntiles for a wave without a tile.
__device__ __forceinline__ int launch_tile(const KArgs &p, int wave)
{
    if (!p.edge_first) return xcd_block() * WAVES_PER_BLOCK + wave;
    const int nb = gridDim.x, b = blockIdx.x, S = p.lead_blocks;
    int lb = b;
    if (b >= S) {  // S is a multiple of 8, so block b still runs on XCD (b - S) mod 8
        const int j = b - S, m8 = (nb - S) & ~7;
        lb = S + ((j < m8) ? ((j & 7) * (m8 >> 3) + (j >> 3)) : j);
    }
    const int i = lb * WAVES_PER_BLOCK + wave;
    if (i >= p.ntiles) return p.ntiles;
    const int tiles_x = p.tiles_x, tiles_y = p.ntiles / tiles_x;
    const int iw = p.txr - p.txl, ih = p.tyb - p.tyt;
    const int nedge = p.ntiles - iw * ih;
    int tx, ty;
    if (i >= nedge) {  // interior, row-major
        const int j = i - nedge;
        ty = p.tyt + j / iw;
        tx = p.txl + j % iw;
    } else {
        const int ntop = p.tyt * tiles_x, nbot = (tiles_y - p.tyb) * tiles_x;
        if (i < ntop) {  // bands above the interior
            ty = i / tiles_x;
            tx = i % tiles_x;
        } else if (i < ntop + nbot) {  // bands below it
            const int j = i - ntop;
            ty = p.tyb + j / tiles_x;
            tx = j % tiles_x;
        } else {  // left and right strips of the interior bands
            const int j = i - ntop - nbot, per = p.txl + (tiles_x - p.txr);
            ty = p.tyt + j / per;
            const int m = j % per;
            tx = m < p.txl ? m : p.txr + (m - p.txl);
        }
    }
    return ty * tiles_x + tx;
}

template <typename T, int V, int K, int RM, int PF, bool VEC>
__global__ __launch_bounds__(WAVE *WAVES_PER_BLOCK) void relax_tb_kernel(const KArgs p)
{
    // the wave index is uniform across the wave; say so, so every tile quantity and
    // every row descriptor lives in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int tile = launch_tile(p, wave);
    if (tile >= p.ntiles) return;  // wave-uniform; waves never synchronise
    const int lane = threadIdx.x & (WAVE - 1);
    unsigned long long rmax = 0;
    double rsum = 0.0;
    relax_one_tile<T, V, K, RM, PF, VEC>(p, tile, lane, rmax, rsum);
    if (RM != RES_NONE) {
        wave_reduce_norms(rmax, rsum, lane);
        if (lane == 0) {
            p.pmax[tile] = rmax;
            p.psum[tile] = rsum;
        }
    }
}

// Batch of independent problems in one persistent launch: the tiles of all
// problems form one list (tile_off = prefix sums of per-problem tile counts) and
// every wave walks it with a stride of the whole grid.  Problems whose `active`
// flag is not 1 are skipped, so a captured launch sequence stays valid while
// problems finish at different times.  Partial norms go to one slot per item.
struct BatchArgs {
    const KArgs *probs;   // per-problem launch arguments (device array)
    const int *tile_off;  // nprob + 1 entries
    const int *active;    // per-problem flag, NULL = all active
    int nprob, total;
    unsigned long long *pmax;
    double *psum;
};

template <typename T, int V, int K, int RM, int PF, bool VEC>
__global__ __launch_bounds__(WAVE *WAVES_PER_BLOCK) void relax_batch_kernel(const BatchArgs b)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (WAVE - 1);
    const int stride = gridDim.x * WAVES_PER_BLOCK;
    for (int item = xcd_block() * WAVES_PER_BLOCK + wave; item < b.total; item += stride) {
        int lo = 0, hi = b.nprob;  // tile_off[lo] <= item < tile_off[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (b.tile_off[mid] <= item) lo = mid; else hi = mid;
        }
        if (b.active && b.active[lo] != 1) continue;
        const KArgs p = b.probs[lo];
        unsigned long long rmax = 0;
        double rsum = 0.0;
        relax_one_tile<T, V, K, RM, PF, VEC>(p, item - b.tile_off[lo], lane, rmax, rsum);
        if (RM != RES_NONE) {
            wave_reduce_norms(rmax, rsum, lane);
            if (lane == 0) {
                b.pmax[item] = rmax;
                b.psum[item] = rsum;
            }
        }
    }
}

using LaunchFn = void (*)(const KArgs &, int, hipStream_t);

template <typename T, int K, int RM, bool VEC>
void launch_inst(const KArgs &ka, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL((relax_tb_kernel<T, VecOf<T>::V, K, RM, PREFETCH, VEC>), dim3(nblocks),
                       dim3(WAVE * WAVES_PER_BLOCK), 0, s, ka);
}

template <typename T, int K, bool VEC>
LaunchFn pick_rm(int rm)
{
    switch (rm) {
    case RES_NONE: return &launch_inst<T, K, RES_NONE, VEC>;
    case RES_LAGGED: return &launch_inst<T, K, RES_LAGGED, VEC>;
    default: return &launch_inst<T, K, RES_FINAL, VEC>;
    }
}

template <typename T, bool VEC>
LaunchFn pick_k(int k, int rm)
{
    switch (k) {
    case 1: return pick_rm<T, 1, VEC>(rm);
    case 2: return pick_rm<T, 2, VEC>(rm);
    case 3: return pick_rm<T, 3, VEC>(rm);
    case 4: return pick_rm<T, 4, VEC>(rm);
    case 5: return pick_rm<T, 5, VEC>(rm);
    case 6: return pick_rm<T, 6, VEC>(rm);
    case 7: return pick_rm<T, 7, VEC>(rm);
    case 8: return pick_rm<T, 8, VEC>(rm);
    default: return nullptr;
    }
}



using BatchLaunchFn = hipError_t (*)(const BatchArgs &, hipStream_t);

// Persistent grid: as many blocks as fit on the device at once.
template <typename T, int K, int RM>
hipError_t launch_batch_inst(const BatchArgs &ba, hipStream_t s)
{
    auto kern = relax_batch_kernel<T, VecOf<T>::V, K, RM, PREFETCH, true>;
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern),
                                                          WAVE * WAVES_PER_BLOCK, 0);
    if (e != hipSuccess) return e;
    const int blocks = std::max(1, std::min(per_cu * cus, (ba.total + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK));
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(WAVE * WAVES_PER_BLOCK), 0, s, ba);
    return hipGetLastError();
}

template <typename T, int K>
BatchLaunchFn pick_batch_rm(int rm)
{
    return rm == RES_NONE ? &launch_batch_inst<T, K, RES_NONE> : &launch_batch_inst<T, K, RES_FINAL>;
}

template <typename T>
BatchLaunchFn pick_batch_k(int k, int rm)
{
    switch (k) {
    case 1: return pick_batch_rm<T, 1>(rm);
    case 2: return pick_batch_rm<T, 2>(rm);
    case 3: return pick_batch_rm<T, 3>(rm);
    case 4: return pick_batch_rm<T, 4>(rm);
    case 5: return pick_batch_rm<T, 5>(rm);
    case 6: return pick_batch_rm<T, 6>(rm);
    case 7: return pick_batch_rm<T, 7>(rm);
    case 8: return pick_batch_rm<T, 8>(rm);
    default: return nullptr;
    }
}

// Per-element-type launcher tables, each compiled in its own translation unit.
BatchLaunchFn pick_batch_f64(int k, int rm);
BatchLaunchFn pick_batch_f32(int k, int rm);
BatchLaunchFn pick_batch_bf16(int k, int rm);
LaunchFn pick_f64(int k, int rm, bool vec);
LaunchFn pick_f32(int k, int rm, bool vec);
LaunchFn pick_bf16(int k, int rm, bool vec);

}  // namespace relax_detail
}  // namespace px
