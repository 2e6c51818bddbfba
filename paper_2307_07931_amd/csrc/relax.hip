// relax.hip -- fused, temporally blocked damped-Jacobi relaxation for gfx950.
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
//     on what the tile itself loaded.  Output columns per wave: `stride`.
// Boundary: DIRICHLET0 replaces the neighbour across the boundary face by
// -(centre) at every level (odd reflection applied on the fly); GHOST_FIXED
// keeps ghost cells as fixed points of every level.
// Results are bit-identical to one sweep at a time: every level rounds to the
// storage type exactly as a store would, and the arithmetic order is fixed:
// s = ((((N - 4C) + W) + E) + S), phi' = (C + w s) - lambda f, r = f - c s.
//
// Partial norms are written per wave (max|r| as bit pattern, sum r^2 in a
// fixed lane/row order) and reduced in fixed order by reduce_partials().
#include "px_internal.h"

#include <algorithm>

namespace px {
namespace {

constexpr int WAVE = 64;
constexpr int WAVES_PER_BLOCK = 4;

template <typename T> struct VecOf;
template <> struct VecOf<double> { static constexpr int V = 2; };
template <> struct VecOf<float> { static constexpr int V = 4; };
template <> struct VecOf<bf16> { static constexpr int V = 4; };

inline int vec_of(int dtype) { return dtype == F64 ? 2 : 4; }

struct Geometry {
    int col_origin, stride, tiles_x, tiles_y, rows, ntiles;
};

// Column partition: output columns [col_origin + tx*stride, ... + stride), the
// origin chosen so that every wave's first loaded column is a multiple of V.
inline Geometry make_geometry(int V, int n, int NL, int rows)
{
    Geometry g;
    const int r = NL % V;
    g.col_origin = (r == 0) ? 0 : r - V;
    const int st = WAVE * V - 2 * NL;
    g.stride = st - st % V;
    g.tiles_x = (n + 2 - g.col_origin + g.stride - 1) / g.stride;
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
    int col_origin, stride, tiles_x, rows, ntiles;
    int phi_vec;  // in/out rows are V-element aligned: vector loads/stores allowed
    int f_vec;    // f rows are aligned so that (column - 1) % V == 0 is a vector
    unsigned long long *pmax;
    double *psum;
};

template <typename T, int V> struct Pack {
    T e[V];
};

// --- cross-lane shifts: lane l receives the value of lane l-1 (up) / l+1 (down).
__device__ __forceinline__ double lane_from_left(double x) { return __shfl_up(x, 1, WAVE); }
__device__ __forceinline__ double lane_from_right(double x) { return __shfl_down(x, 1, WAVE); }
__device__ __forceinline__ float lane_from_left(float x) { return __shfl_up(x, 1, WAVE); }
__device__ __forceinline__ float lane_from_right(float x) { return __shfl_down(x, 1, WAVE); }

// Load V consecutive elements of row `row` (columns col0..col0+V-1) of an
// array with `nrows` rows of `ld` elements; anything outside reads as 0.
template <typename T, int V>
__device__ __forceinline__ void load_row(const T *__restrict__ base, int row, int nrows, int ld,
                                         int col0, bool vec_ok, typename Elem<T>::A (&dst)[V])
{
    using E = Elem<T>;
    if (row < 0 || row >= nrows) {
#pragma unroll
        for (int v = 0; v < V; ++v) dst[v] = 0;
        return;
    }
    const T *rp = base + (size_t)row * (size_t)ld;
    if (vec_ok && col0 >= 0 && col0 + V <= ld) {
        const Pack<T, V> pk = *reinterpret_cast<const Pack<T, V> *>(rp + col0);
#pragma unroll
        for (int v = 0; v < V; ++v) dst[v] = E::load(pk.e[v]);
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int c = col0 + v;
            dst[v] = (c >= 0 && c < ld) ? E::load(rp[c]) : (typename Elem<T>::A)0;
        }
    }
}

// Store the elements of V consecutive columns that fall in [lo, hi).
template <typename T, int V>
__device__ __forceinline__ void store_row(T *__restrict__ rp, int col0, int lo, int hi, bool vec_ok,
                                          const typename Elem<T>::A (&val)[V], bool negate)
{
    using E = Elem<T>;
    if (vec_ok && col0 >= lo && col0 + V <= hi) {
        Pack<T, V> pk;
#pragma unroll
        for (int v = 0; v < V; ++v) pk.e[v] = E::store(negate ? -val[v] : val[v]);
        *reinterpret_cast<Pack<T, V> *>(rp + col0) = pk;
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int c = col0 + v;
            if (c >= lo && c < hi) rp[c] = E::store(negate ? -val[v] : val[v]);
        }
    }
}

template <typename T, int V, int K, int RM>
__global__ __launch_bounds__(WAVE *WAVES_PER_BLOCK) void relax_tb_kernel(const KArgs p)
{
    using E = Elem<T>;
    using A = typename E::A;
    constexpr int NL = K + (RM == RES_FINAL ? 1 : 0);  // pipeline levels
    constexpr int RL = (RM == RES_FINAL) ? K + 1 : K;  // level that takes the residual
    constexpr int FQ = RL + 1;                         // f rows kept in flight

    // XCD-aware block order: block b runs on XCD b % 8; give each XCD a contiguous
    // run of tiles so neighbouring tiles (shared halo rows/columns) share an L2.
    const int nb = gridDim.x, b = blockIdx.x;
    const int nb8 = nb & ~7;
    const int lb = (b < nb8) ? ((b & 7) * (nb8 >> 3) + (b >> 3)) : b;
    const int tile = lb * WAVES_PER_BLOCK + (threadIdx.x >> 6);
    if (tile >= p.ntiles) return;  // wave-uniform; waves never synchronise
    const int lane = threadIdx.x & (WAVE - 1);

    const int n = p.n;
    const int tx = tile % p.tiles_x, ty = tile / p.tiles_x;
    const int oc0 = p.col_origin + tx * p.stride;  // output columns [oc0, oc1)
    const int oc1 = min(oc0 + p.stride, n + 2);
    const int mc = oc0 - NL + lane * V;            // first column held by this lane
    const int y0 = ty * p.rows, y1 = min(y0 + p.rows, n + 2);

    const A w = (A)p.w, cc = (A)p.c, lam = (A)p.lam;
    const bool dir = (p.bc == DIRICHLET0);
    const bool pv = p.phi_vec != 0, fv = p.f_vec != 0;
    const T *__restrict__ in = static_cast<const T *>(p.in);
    const T *__restrict__ fp = static_cast<const T *>(p.f);
    T *__restrict__ out = static_cast<T *>(p.out);

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

    unsigned long long rmax = 0;
    double rsum = 0.0;
    // residual window of this wave: rows [ry0, ry1), columns [rc0, rc1), interior only
    const int ry0 = max(y0, 1), ry1 = min(y1, n + 1);
    const int rc0 = max(oc0, 1), rc1 = min(oc1, n + 1);

    for (int s = y0 - NL; s < y1 + NL; ++s) {
        // ---- level 0: input row s and f of row s
#pragma unroll
        for (int v = 0; v < V; ++v) {
            win[0][0][v] = win[0][1][v];
            win[0][1][v] = win[0][2][v];
        }
        load_row<T, V>(in, s, n + 2, p.ld, mc, pv, win[0][2]);
#pragma unroll
        for (int j = FQ - 1; j > 0; --j)
#pragma unroll
            for (int v = 0; v < V; ++v) fq[j][v] = fq[j - 1][v];
        if (s >= 1 && s <= n) {
            load_row<T, V>(fp, s - 1, n, p.ld_f, mc - 1, fv, fq[0]);
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) fq[0][v] = 0;
        }

        // ---- levels 1..NL, level t at row s - t
#pragma unroll
        for (int t = 1; t <= NL; ++t) {
            if (s < y0 - NL + 2 * t) break;  // rows this level does not need yet
            const int r = s - t;
            const A left = lane_from_left(win[t - 1][1][V - 1]);
            const A right = lane_from_right(win[t - 1][1][0]);
            A st[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const A C = win[t - 1][1][v];
                A N = win[t - 1][0][v];
                A S = win[t - 1][2][v];
                A Wn = (v == 0) ? left : win[t - 1][1][v - 1];
                A En = (v == V - 1) ? right : win[t - 1][1][v + 1];
                if (dir) {
                    const int col = mc + v;
                    if (r == 1) N = -C;
                    if (r == n) S = -C;
                    if (col == 1) Wn = -C;
                    if (col == n) En = -C;
                }
                st[v] = (((N - (A)4 * C) + Wn) + En) + S;
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
                    nv[v] = inter ? u : (dir ? (A)0 : C);
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
                    T *rp = out + (size_t)r * (size_t)p.ld;
                    if (dir) {
                        if (row_in) {
                            store_row<T, V>(rp, mc, rc0, rc1, pv, nv, false);
                            // edge ghosts of this row and, on rows 1 and n, the ghost rows
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                const int col = mc + v;
                                if (col >= rc0 && col < rc1) {
                                    if (col == 1) rp[0] = E::store(-nv[v]);
                                    if (col == n) rp[n + 1] = E::store(-nv[v]);
                                }
                            }
                            if (r == 1) store_row<T, V>(out, mc, rc0, rc1, false, nv, true);
                            if (r == n)
                                store_row<T, V>(out + (size_t)(n + 1) * (size_t)p.ld, mc, rc0, rc1,
                                                false, nv, true);
                        }
                    } else {
                        const bool ghost_row = (r == 0 || r == n + 1);
                        const int lo = max(oc0, ghost_row ? 1 : 0);
                        const int hi = min(oc1, ghost_row ? n + 1 : n + 2);
                        store_row<T, V>(rp, mc, lo, hi, pv, nv, false);
                    }
                }
            }
            if (RM != RES_NONE && t == RL && r >= ry0 && r < ry1) {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int col = mc + v;
                    if (col >= rc0 && col < rc1) {
                        const A rr = fq[t][v] - cc * st[v];
                        const double rd = (double)rr;
                        const unsigned long long bits =
                            (unsigned long long)__double_as_longlong(fabs(rd));
                        rmax = bits > rmax ? bits : rmax;
                        rsum += rd * rd;
                    }
                }
            }
        }
    }

    if (RM != RES_NONE) {
#pragma unroll
        for (int off = WAVE / 2; off > 0; off >>= 1) {
            const unsigned long long om = __shfl_xor(rmax, off, WAVE);
            const double os = __shfl_xor(rsum, off, WAVE);
            rmax = om > rmax ? om : rmax;
            // fixed pairing: the lower lane's value always comes first
            rsum = (lane & off) ? (os + rsum) : (rsum + os);
        }
        if (lane == 0) {
            p.pmax[tile] = rmax;
            p.psum[tile] = rsum;
        }
    }
}

using LaunchFn = void (*)(const KArgs &, int, hipStream_t);

template <typename T, int K, int RM>
void launch_inst(const KArgs &ka, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL((relax_tb_kernel<T, VecOf<T>::V, K, RM>), dim3(nblocks),
                       dim3(WAVE * WAVES_PER_BLOCK), 0, s, ka);
}

template <typename T, int K>
LaunchFn pick_rm(int rm)
{
    switch (rm) {
    case RES_NONE: return &launch_inst<T, K, RES_NONE>;
    case RES_LAGGED: return &launch_inst<T, K, RES_LAGGED>;
    default: return &launch_inst<T, K, RES_FINAL>;
    }
}

template <typename T>
LaunchFn pick_k(int k, int rm)
{
    switch (k) {
    case 1: return pick_rm<T, 1>(rm);
    case 2: return pick_rm<T, 2>(rm);
    case 3: return pick_rm<T, 3>(rm);
    case 4: return pick_rm<T, 4>(rm);
    case 5: return pick_rm<T, 5>(rm);
    case 6: return pick_rm<T, 6>(rm);
    case 7: return pick_rm<T, 7>(rm);
    case 8: return pick_rm<T, 8>(rm);
    default: return nullptr;
    }
}

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace

int relax_default_rows(int dtype, int n, int sweeps)
{
    (void)dtype;
    // Enough tiles to give every SIMD several waves, long enough bands that the
    // recomputed halo rows (about sweeps/rows) stay small.
    int rows = sweeps <= 1 ? 32 : sweeps <= 2 ? 64 : 128;
    const int cap = std::max(8, (n + 2) / 8);
    return std::min(rows, cap);
}

int relax_num_waves(int dtype, int n, int sweeps, int resmode, int rows)
{
    const int NL = sweeps + (resmode == RES_FINAL ? 1 : 0);
    return make_geometry(vec_of(dtype), n, NL, rows).ntiles;
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
    ka.col_origin = g.col_origin;
    ka.stride = g.stride;
    ka.tiles_x = g.tiles_x;
    ka.rows = g.rows;
    ka.ntiles = g.ntiles;
    ka.phi_vec = (aligned(a.in, V * es) && aligned(a.out, V * es) && a.ld % V == 0) ? 1 : 0;
    // f column (c-1) is vector aligned when c % V == 0: needs (f - 1 element) aligned
    ka.f_vec = (aligned(static_cast<const char *>(a.f) - es, V * es) && a.ld_f % V == 0) ? 1 : 0;
    ka.pmax = a.part.max_bits;
    ka.psum = a.part.sum;
    LaunchFn fn = nullptr;
    switch (dtype) {
    case F64: fn = pick_k<double>(a.sweeps, a.resmode); break;
    case F32: fn = pick_k<float>(a.sweeps, a.resmode); break;
    case BF16: fn = pick_k<bf16>(a.sweeps, a.resmode); break;
    }
    if (!fn) return hipErrorInvalidValue;
    const int nblocks = (g.ntiles + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
    fn(ka, nblocks, s);
    return hipGetLastError();
}

}  // namespace px
