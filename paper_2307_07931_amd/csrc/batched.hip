// batched.hip -- many independent Poisson problems at once.
//
// Relaxation: the tiles of every problem form one work list walked by one
// persistent launch per k sweeps (relax_batch_kernel in relax_kernel.h).
// Solve: FP64 iterative refinement around FP32/BF16 inner sweeps, the same
// arithmetic as the single-problem solve.  One outer step for the whole batch
// is a fixed sequence of launches -- zero the corrections, the inner sweeps,
// the FP64 residual/update, per-problem norms, a convergence check -- captured
// once in a hipGraph and replayed.  Which problems still run is decided on the
// device: the check switches a converged problem's flag off and every kernel
// skips it, so the captured graph never changes.  Each problem's FP64 iterate
// alternates between the caller's buffer and a twin (a per-problem parity bit
// flipped by the check kernel).
#include "../../include/protox.h"
#include "px_internal.h"
#include "relax_kernel.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

namespace px {
using namespace relax_detail;

namespace {

constexpr int BX = 256;

// ------------------------------------------------------------------ kernels

// Problem owning flat item `item` given prefix sums off[0..nprob].
__device__ __forceinline__ int owner(const int *off, int nprob, int item)
{
    int lo = 0, hi = nprob;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void block_reduce_norms(unsigned long long &mx, double &sm)
{
    __shared__ unsigned long long smx[BX / 64];
    __shared__ double ssm[BX / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long om = __shfl_xor(mx, off, 64);
        const double os = __shfl_xor(sm, off, 64);
        mx = om > mx ? om : mx;
        sm = (lane & off) ? (os + sm) : (sm + os);
    }
    if (lane == 0) {
        smx[wv] = mx;
        ssm[wv] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = smx[0];
        sm = ssm[0];
        for (int k = 1; k < BX / 64; ++k) {
            mx = smx[k] > mx ? smx[k] : mx;
            sm = sm + ssm[k];
        }
    }
}

// Per-problem refinement data (FP64 iterate in two buffers, low-precision correction
// and right-hand side of the inner solve).
struct RefineProb {
    double *phi[2];
    const void *delta;  // final correction of the inner sweeps (ld_l)
    const double *f;
    void *r_low;        // n x ld_l
    void *zero;         // the correction buffer the inner sweeps start from (ld_l)
    int n, ld, ld_f, ld_l, bc;
    double c;
};

struct RowArgs {
    const RefineProb *probs;
    const int *row_off;  // prefix sums of n over problems
    int nprob, total_rows;
    const int *active;
    const int *parity;
    int use_delta;
    unsigned long long *pmax;  // one slot per row
    double *psum;
};

// FP64 outer step for one row of one problem: phi_out = phi_in + delta, r = f - L phi_out,
// r rounded into r_low, partial norms of r.  Same arithmetic as refine_kernel.
template <typename L>
__global__ __launch_bounds__(BX) void refine_rows_kernel(const RowArgs a)
{
    const int row = blockIdx.x;
    const int p = owner(a.row_off, a.nprob, row);
    unsigned long long mx = 0;
    double sm = 0.0;
    const bool on = a.active[p] == 1;
    if (on) {
        const RefineProb q = a.probs[p];
        const int i = row - a.row_off[p] + 1, n = q.n, ld = q.ld;
        const int par = a.parity[p];
        const double *phi_in = q.phi[par];
        double *phi_out = q.phi[1 - par];
        const L *delta = a.use_delta ? static_cast<const L *>(q.delta) : nullptr;
        const bool dir = q.bc == DIRICHLET0;
        auto upd = [&](int ii, int jj) -> double {
            double v = phi_in[(size_t)ii * ld + jj];
            if (delta && ii >= 1 && ii <= n && jj >= 1 && jj <= n)
                v = v + (double)Elem<L>::load(delta[(size_t)ii * q.ld_l + jj]);
            return v;
        };
        for (int j = threadIdx.x + 1; j <= n; j += BX) {
            const double C = upd(i, j);
            const double N = (dir && i == 1) ? -C : upd(i - 1, j);
            const double W = (dir && j == 1) ? -C : upd(i, j - 1);
            const double E = (dir && j == n) ? -C : upd(i, j + 1);
            const double S = (dir && i == n) ? -C : upd(i + 1, j);
            const double s = (((N - 4.0 * C) + W) + E) + S;
            const double rr = q.f[(size_t)(i - 1) * q.ld_f + (j - 1)] - q.c * s;
            phi_out[(size_t)i * ld + j] = C;
            if (dir) {
                if (i == 1) phi_out[j] = -C;
                if (i == n) phi_out[(size_t)(n + 1) * ld + j] = -C;
                if (j == 1) phi_out[(size_t)i * ld] = -C;
                if (j == n) phi_out[(size_t)i * ld + n + 1] = -C;
            } else {
                if (i == 1) phi_out[j] = phi_in[j];
                if (i == n) phi_out[(size_t)(n + 1) * ld + j] = phi_in[(size_t)(n + 1) * ld + j];
                if (j == 1) phi_out[(size_t)i * ld] = phi_in[(size_t)i * ld];
                if (j == n) phi_out[(size_t)i * ld + n + 1] = phi_in[(size_t)i * ld + n + 1];
            }
            static_cast<L *>(q.r_low)[(size_t)(i - 1) * q.ld_l + (j - 1)] = Elem<L>::store((float)rr);
            const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(rr));
            mx = b > mx ? b : mx;
            sm = sm + rr * rr;
        }
    }
    block_reduce_norms(mx, sm);
    if (threadIdx.x == 0) {
        a.pmax[row] = mx;
        a.psum[row] = sm;
    }
}

// max|f| and sum f^2 of one row (partials per row slot).
__global__ __launch_bounds__(BX) void fnorm_rows_kernel(const RowArgs a)
{
    const int row = blockIdx.x;
    const int p = owner(a.row_off, a.nprob, row);
    const RefineProb q = a.probs[p];
    const int i = row - a.row_off[p];
    unsigned long long mx = 0;
    double sm = 0.0;
    for (int j = threadIdx.x; j < q.n; j += BX) {
        const double v = q.f[(size_t)i * q.ld_f + j];
        const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(v));
        mx = b > mx ? b : mx;
        sm = sm + v * v;
    }
    block_reduce_norms(mx, sm);
    if (threadIdx.x == 0) {
        a.pmax[row] = mx;
        a.psum[row] = sm;
    }
}

// Zero the starting correction (ghost ring included) of active problems; one grid row
// (n + 2 of them per problem, rows counted by row_off over n + 2) per block.
template <typename L>
__global__ __launch_bounds__(BX) void zero_rows_kernel(const RowArgs a)
{
    const int row = blockIdx.x;
    const int p = owner(a.row_off, a.nprob, row);
    if (a.active[p] != 1) return;
    const RefineProb q = a.probs[p];
    const int i = row - a.row_off[p];
    L *z = static_cast<L *>(q.zero);
    for (int j = threadIdx.x; j < q.ld_l; j += BX) z[(size_t)i * q.ld_l + j] = L{};
}

// FP64 iterate back into the caller's buffer for problems whose parity ended at 1.
__global__ __launch_bounds__(BX) void copyback_rows_kernel(const RowArgs a)
{
    const int row = blockIdx.x;
    const int p = owner(a.row_off, a.nprob, row);
    if (a.parity[p] != 1) return;
    const RefineProb q = a.probs[p];
    const int i = row - a.row_off[p];
    const int n = q.n;
    for (int j = threadIdx.x; j <= n + 1; j += BX) {
        if ((i == 0 || i == n + 1) && (j == 0 || j == n + 1)) continue;
        q.phi[0][(size_t)i * q.ld + j] = q.phi[1][(size_t)i * q.ld + j];
    }
}

// Result of an odd number of relaxation launches back into the callers' grids, all
// problems in one launch: block (x, p) copies rows x, x + gridDim.x, ... of problem p
// from args[p].out to args[p].in (corners untouched, as by every relaxation).
template <typename T>
__global__ __launch_bounds__(BX) void copy_back_kernel(const KArgs *args)
{
    const KArgs q = args[blockIdx.y];
    const int n = q.n;
    const T *src = static_cast<const T *>(q.out);
    T *dst = static_cast<T *>(const_cast<void *>(q.in));
    for (int i = blockIdx.x; i <= n + 1; i += gridDim.x)
        for (int j = threadIdx.x; j <= n + 1; j += BX) {
            if ((i == 0 || i == n + 1) && (j == 0 || j == n + 1)) continue;
            dst[(size_t)i * q.ld + j] = src[(size_t)i * q.ld + j];
        }
}

hipError_t copy_back_launch(int dtype, const KArgs *args, int nprob, hipStream_t s)
{
    const dim3 g(64, nprob);
    switch (dtype) {
    case F64: hipLaunchKernelGGL((copy_back_kernel<double>), g, dim3(BX), 0, s, args); break;
    case F32: hipLaunchKernelGGL((copy_back_kernel<float>), g, dim3(BX), 0, s, args); break;
    case BF16: hipLaunchKernelGGL((copy_back_kernel<bf16>), g, dim3(BX), 0, s, args); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Per-problem fixed-order reduction of contiguous partial slots [off[p], off[p+1]).
__global__ __launch_bounds__(BX) void reduce_per_problem_kernel(const unsigned long long *pmax,
                                                                const double *psum, const int *off,
                                                                const int *active, double *norms)
{
    const int p = blockIdx.x;
    if (active && active[p] != 1) return;
    unsigned long long mx = 0;
    double sm = 0.0;
    for (int k = off[p] + threadIdx.x; k < off[p + 1]; k += BX) {
        mx = pmax[k] > mx ? pmax[k] : mx;
        sm = sm + psum[k];
    }
    block_reduce_norms(mx, sm);
    if (threadIdx.x == 0) {
        norms[2 * p] = __longlong_as_double((long long)mx);
        norms[2 * p + 1] = sm;
    }
}

// Convergence state per problem.
enum { ST_RUN = 1, ST_DONE = 0, ST_BUDGET = -1, ST_NONFINITE = -2, ST_DIVERGED = -3 };

struct CheckArgs {
    int nprob;
    int *active, *parity;
    long long *steps, *sweeps;
    const double *norms;    // 2 per problem
    const double *fnorms;   // 2 per problem: max|f|, sum f^2
    double *r0;             // first residual measure per problem
    int use_l2;
    double rtol;
    long long max_sweeps;
    int inner;              // sweeps of the step just done (0 for the first check)
};

__global__ __launch_bounds__(BX) void check_kernel(const CheckArgs a)
{
    const int p = blockIdx.x * BX + threadIdx.x;
    if (p >= a.nprob || a.active[p] != ST_RUN) return;
    a.parity[p] ^= 1;  // this step's refinement wrote the other buffer
    const double mx = a.norms[2 * p], sq = a.norms[2 * p + 1];
    const double m = a.use_l2 ? sqrt(sq) : mx;
    const double fref = a.use_l2 ? sqrt(a.fnorms[2 * p + 1]) : a.fnorms[2 * p];
    if (a.inner == 0) a.r0[p] = m;
    else {
        a.steps[p] += 1;
        a.sweeps[p] += a.inner;
    }
    if (!isfinite(mx) || !isfinite(sq)) a.active[p] = ST_NONFINITE;
    else if (m <= a.rtol * fref) a.active[p] = ST_DONE;
    else if (m > 1e8 * fmax(a.r0[p], fref)) a.active[p] = ST_DIVERGED;
    else if (a.sweeps[p] >= a.max_sweeps) a.active[p] = ST_BUDGET;
}

template <typename T> T *dev_ptr(char *base, size_t off) { return reinterpret_cast<T *>(base + off); }

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

BatchLaunchFn pick_batch(int dtype, int k, int rm)
{
    switch (dtype) {
    case F64: return pick_batch_f64(k, rm);
    case F32: return pick_batch_f32(k, rm);
    case BF16: return pick_batch_bf16(k, rm);
    default: return nullptr;
    }
}

// Launch arguments of one problem (geometry for k sweeps per launch and tile rows).
KArgs make_kargs(int dtype, const void *in, void *out, const void *f, int n, int ld, int ld_f, double h,
                 double lambda, int bc, int k, int rm, int rows)
{
    const int V = dtype == F64 ? 2 : 4;
    const int NL = k + (rm == RES_FINAL ? 1 : 0);
    const Geometry g = make_geometry(V, n, NL, rows);  // the kernel assumes this geometry
    KArgs a;
    std::memset(&a, 0, sizeof a);
    a.in = in;
    a.out = out;
    a.f = f;
    a.n = n;
    a.ld = ld;
    a.ld_f = ld_f;
    a.bc = bc;
    a.c = 1.0 / (h * h);
    a.w = lambda / (h * h);
    a.lam = lambda;
    a.halo = g.halo;
    a.col_origin = g.col_origin;
    a.stride = g.stride;
    a.tiles_x = g.tiles_x;
    a.rows = g.rows;
    a.ntiles = g.ntiles;
    return a;
}

}  // namespace

int BatchWork::rows_for(int dtype, int n, int k, int forced) const
{
    if (forced > 0) return forced;
    for (const auto &e : tuned_rows[dtype])
        if (e.first == n) return e.second;
    return relax_default_rows(dtype, n, k);
}

// ---------------------------------------------------------- scratch memory

BatchWork::~BatchWork()
{
    if (mem) (void)hipFree(mem);
    if (graph_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph_exec));
    if (stream) (void)hipStreamDestroy(static_cast<hipStream_t>(stream));
}

hipError_t BatchWork::ensure(size_t need)
{
    if (bytes >= need) return hipSuccess;
    if (mem) (void)hipFree(mem);
    mem = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&mem, need);
    if (e == hipSuccess) bytes = need;
    return e;
}

// ------------------------------------------------------------- relaxation

int batch_relax(BatchWork &w, int dtype, const BatchProblem *probs, int nprob, int nsweeps, int k, int bc,
                int resmode, double *norms, int forced_rows, hipStream_t s, char *err, size_t errlen)
{
    const size_t es = (size_t)elem_size(dtype);
    const int L = (nsweeps + k - 1) / k;
    // layout: tmp grids | 3 arg arrays per launch size (k, remainder) | tile offsets | partials
    std::vector<size_t> tmp_off(nprob);
    size_t off = 0;
    for (int p = 0; p < nprob; ++p) {
        tmp_off[p] = off;
        off += round256((size_t)(probs[p].n + 2) * probs[p].ld * es);
    }
    const int krem = nsweeps - (L - 1) * k;  // sweeps of the last launch
    // per distinct launch shape (k, rm) the tile offsets and three argument arrays:
    // [0] phi -> tmp, [1] tmp -> phi, both with that shape
    struct Shape {
        int k, rm;
        size_t args_off[2], toff_off;
        int total;
        std::vector<KArgs> a[2];
        std::vector<int> toff;
    };
    std::vector<Shape> shapes;
    auto shape_of = [&](int kk, int rm) -> int {
        for (size_t i = 0; i < shapes.size(); ++i)
            if (shapes[i].k == kk && shapes[i].rm == rm) return (int)i;
        Shape sh;
        sh.k = kk;
        sh.rm = rm;
        sh.toff.assign(nprob + 1, 0);
        for (int dir = 0; dir < 2; ++dir) sh.a[dir].resize(nprob);
        for (int p = 0; p < nprob; ++p) {
            const BatchProblem &q = probs[p];
            const int rows = w.rows_for(dtype, q.n, kk, forced_rows);
            char *tmp = nullptr;  // filled after allocation
            sh.a[0][p] = make_kargs(dtype, q.phi, tmp, q.f, q.n, q.ld, q.ld_f, q.h, q.lambda, bc, kk, rm, rows);
            sh.a[1][p] = make_kargs(dtype, tmp, q.phi, q.f, q.n, q.ld, q.ld_f, q.h, q.lambda, bc, kk, rm, rows);
            sh.toff[p + 1] = sh.toff[p] + sh.a[0][p].ntiles;
        }
        sh.total = sh.toff[nprob];
        shapes.push_back(std::move(sh));
        return (int)shapes.size() - 1;
    };
    std::vector<int> seq(L);
    for (int i = 0; i < L; ++i) {
        const int kk = (i == L - 1) ? krem : k;
        const int rm = (i == L - 1 && resmode != RES_NONE) ? RES_FINAL : RES_NONE;
        seq[i] = shape_of(kk, rm);
    }
    size_t parts = 0;
    for (auto &sh : shapes) {
        for (int dir = 0; dir < 2; ++dir) {
            sh.args_off[dir] = off;
            off += round256(sizeof(KArgs) * nprob);
        }
        sh.toff_off = off;
        off += round256(sizeof(int) * (nprob + 1));
        parts = std::max(parts, (size_t)sh.total);
    }
    const size_t pmax_off = off;
    off += round256(parts * 8);
    const size_t psum_off = off;
    off += round256(parts * 8);
    hipError_t e = w.ensure(off);
    if (e != hipSuccess) {
        snprintf(err, errlen, "hipMalloc(%zu) for the batch failed", off);
        return PX_ENOMEM;
    }
    char *base = static_cast<char *>(w.mem);
    for (auto &sh : shapes) {
        for (int p = 0; p < nprob; ++p) {
            sh.a[0][p].out = base + tmp_off[p];
            sh.a[1][p].in = base + tmp_off[p];
        }
        for (int dir = 0; dir < 2; ++dir)
            if ((e = hipMemcpyAsync(base + sh.args_off[dir], sh.a[dir].data(), sizeof(KArgs) * nprob,
                                    hipMemcpyHostToDevice, s)) != hipSuccess)
                break;
        if (e == hipSuccess)
            e = hipMemcpyAsync(base + sh.toff_off, sh.toff.data(), sizeof(int) * (nprob + 1),
                               hipMemcpyHostToDevice, s);
        if (e != hipSuccess) break;
    }
    for (int i = 0; i < L && e == hipSuccess; ++i) {
        const Shape &sh = shapes[seq[i]];
        BatchArgs ba;
        ba.probs = dev_ptr<const KArgs>(base, sh.args_off[i % 2]);
        ba.tile_off = dev_ptr<const int>(base, sh.toff_off);
        ba.active = nullptr;
        ba.nprob = nprob;
        ba.total = sh.total;
        ba.pmax = dev_ptr<unsigned long long>(base, pmax_off);
        ba.psum = dev_ptr<double>(base, psum_off);
        BatchLaunchFn fn = pick_batch(dtype, sh.k, sh.rm);
        if (!fn) e = hipErrorInvalidValue;
        else e = fn(ba, s);
        if (e == hipSuccess && sh.rm != RES_NONE) {
            hipLaunchKernelGGL(reduce_per_problem_kernel, dim3(nprob), dim3(BX), 0, s, ba.pmax, ba.psum,
                               ba.tile_off, (const int *)nullptr, norms);
            e = hipGetLastError();
        }
    }
    // an odd number of launches leaves the result in the scratch grids: copy it back
    // (the phi -> scratch arguments of any shape name both grids of every problem)
    if (e == hipSuccess && L % 2 == 1)
        e = copy_back_launch(dtype, dev_ptr<const KArgs>(base, shapes[seq[0]].args_off[0]), nprob, s);
    if (e != hipSuccess) {
        snprintf(err, errlen, "batched relaxation: %s", hipGetErrorString(e));
        return PX_EHIP;
    }
    return PX_OK;
}

// ------------------------------------------------------------ multi-box domains

namespace {

struct BoxDesc {
    void *phi;
    int ld, pad;
};

template <typename T> __device__ __forceinline__ T negated(T x) { return -x; }
template <> __device__ __forceinline__ bf16 negated(bf16 x) { return bf16{(unsigned short)(x.bits ^ 0x8000u)}; }

// One ghost cell per thread: blockIdx.z = box, blockIdx.y = side (0 north: row 0, 1 south:
// row n + 1, 2 west: column 0, 3 east: column n + 1), index 1..n along the side.  A side
// facing another box copies that box's adjacent interior row or column; a side on the
// domain edge takes -(adjacent interior) under DIRICHLET0, wraps onto the opposite box
// under PERIODIC, and is left alone under GHOST_FIXED.  Only ghost cells are written and
// only interior cells read, so the boxes can be refreshed all at once.  Corners are not
// touched (the 5-point stencil does not read them).
template <typename T>
__global__ __launch_bounds__(BX) void box_exchange_kernel(const BoxDesc *__restrict__ boxes, int nbx, int nby, int n,
                                                          int bc)
{
    const int idx = (int)(blockIdx.x * BX + threadIdx.x) + 1;
    if (idx > n) return;
    const int side = (int)blockIdx.y, b = (int)blockIdx.z;
    const int bi = b / nbx, bj = b % nbx;
    T *me = static_cast<T *>(boxes[b].phi);
    const size_t ld = (size_t)boxes[b].ld;
    int ni = bi, nj = bj;  // the box across this side
    if (side == 0) ni = bi - 1;
    else if (side == 1) ni = bi + 1;
    else if (side == 2) nj = bj - 1;
    else nj = bj + 1;
    const bool inside = ni >= 0 && ni < nby && nj >= 0 && nj < nbx;
    // ghost position and the interior cell it mirrors, in this box
    size_t g, a;
    if (side == 0) { g = (size_t)idx; a = ld + idx; }
    else if (side == 1) { g = (size_t)(n + 1) * ld + idx; a = (size_t)n * ld + idx; }
    else if (side == 2) { g = (size_t)idx * ld; a = (size_t)idx * ld + 1; }
    else { g = (size_t)idx * ld + n + 1; a = (size_t)idx * ld + n; }
    if (!inside && bc == PERIODIC) {
        ni = (ni + nby) % nby;
        nj = (nj + nbx) % nbx;
    } else if (!inside) {
        if (bc == DIRICHLET0) me[g] = negated(me[a]);
        return;
    }
    const T *nb = static_cast<const T *>(boxes[ni * nbx + nj].phi);
    const size_t ldn = (size_t)boxes[ni * nbx + nj].ld;
    size_t src;  // the neighbour's interior cell next to this ghost
    if (side == 0) src = (size_t)n * ldn + idx;
    else if (side == 1) src = ldn + idx;
    else if (side == 2) src = (size_t)idx * ldn + n;
    else src = (size_t)idx * ldn + 1;
    me[g] = nb[src];
}

}  // namespace

// Periods of `exchange` sweeps alternate between the boxes' own grids and scratch grids: one
// exchange launch on the current grids, then one persistent relaxation launch into the
// other set (fixed ghosts: each box's ghost ring travels with it); launch arguments and box
// descriptors of both directions are uploaded once, and an odd number of periods ends with
// one copy of every result back.
int batch_relax_boxes(BatchWork &w, int dtype, const BatchProblem *probs, int nbx, int nby, int nsweeps, int exchange,
                      int bc, int forced_rows, hipStream_t s, char *err, size_t errlen)
{
    const int nbox = nbx * nby, n = probs[0].n;
    const int periods = nsweeps / exchange;
    if (periods == 0) return PX_OK;
    const size_t es = (size_t)elem_size(dtype);
    // layout: scratch grids | launch arguments [2][nbox] | tile offsets | box descriptors [2][nbox]
    std::vector<size_t> tmp_off(nbox);
    size_t off = 0;
    for (int b = 0; b < nbox; ++b) {
        tmp_off[b] = off;
        off += round256((size_t)(n + 2) * probs[b].ld * es);
    }
    const size_t args_off[2] = {off, off + round256(sizeof(KArgs) * nbox)};
    off = args_off[1] + round256(sizeof(KArgs) * nbox);
    const size_t toff_off = off;
    off += round256(sizeof(int) * (nbox + 1));
    const size_t desc_off[2] = {off, off + round256(sizeof(BoxDesc) * nbox)};
    off = desc_off[1] + round256(sizeof(BoxDesc) * nbox);
    hipError_t e = w.ensure(off);
    if (e != hipSuccess) {
        snprintf(err, errlen, "hipMalloc(%zu) for the boxes failed", off);
        return PX_ENOMEM;
    }
    char *base = static_cast<char *>(w.mem);
    std::vector<KArgs> a[2];
    std::vector<BoxDesc> d[2];
    std::vector<int> toff(nbox + 1, 0);
    for (int dir = 0; dir < 2; ++dir) {
        a[dir].resize(nbox);
        d[dir].resize(nbox);
    }
    for (int b = 0; b < nbox; ++b) {
        const BatchProblem &q = probs[b];
        void *tmp = base + tmp_off[b];
        const int rows = w.rows_for(dtype, n, exchange, forced_rows);
        a[0][b] = make_kargs(dtype, q.phi, tmp, q.f, n, q.ld, q.ld_f, q.h, q.lambda, GHOST_FIXED, exchange, RES_NONE,
                             rows);
        a[1][b] = make_kargs(dtype, tmp, q.phi, q.f, n, q.ld, q.ld_f, q.h, q.lambda, GHOST_FIXED, exchange, RES_NONE,
                             rows);
        toff[b + 1] = toff[b] + a[0][b].ntiles;
        d[0][b] = BoxDesc{q.phi, q.ld, 0};
        d[1][b] = BoxDesc{tmp, q.ld, 0};
    }
    for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
        e = hipMemcpyAsync(base + args_off[dir], a[dir].data(), sizeof(KArgs) * nbox, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(base + desc_off[dir], d[dir].data(), sizeof(BoxDesc) * nbox, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + toff_off, toff.data(), sizeof(int) * (nbox + 1), hipMemcpyHostToDevice, s);
    BatchLaunchFn fn = pick_batch(dtype, exchange, RES_NONE);
    if (!fn && e == hipSuccess) e = hipErrorInvalidValue;
    const dim3 grid((unsigned)((n + BX - 1) / BX), 4u, (unsigned)nbox);
    for (int i = 0; i < periods && e == hipSuccess; ++i) {
        const BoxDesc *cur = dev_ptr<const BoxDesc>(base, desc_off[i % 2]);
        switch (dtype) {
        case F64: hipLaunchKernelGGL(box_exchange_kernel<double>, grid, dim3(BX), 0, s, cur, nbx, nby, n, bc); break;
        case F32: hipLaunchKernelGGL(box_exchange_kernel<float>, grid, dim3(BX), 0, s, cur, nbx, nby, n, bc); break;
        default: hipLaunchKernelGGL(box_exchange_kernel<bf16>, grid, dim3(BX), 0, s, cur, nbx, nby, n, bc); break;
        }
        if ((e = hipGetLastError()) != hipSuccess) break;
        BatchArgs ba;
        ba.probs = dev_ptr<const KArgs>(base, args_off[i % 2]);
        ba.tile_off = dev_ptr<const int>(base, toff_off);
        ba.active = nullptr;
        ba.nprob = nbox;
        ba.total = toff[nbox];
        ba.pmax = nullptr;  // no norms
        ba.psum = nullptr;
        e = fn(ba, s);
    }
    if (e == hipSuccess && periods % 2 == 1)
        e = copy_back_launch(dtype, dev_ptr<const KArgs>(base, args_off[0]), nbox, s);
    if (e != hipSuccess) {
        snprintf(err, errlen, "box relaxation: %s", hipGetErrorString(e));
        return PX_EHIP;
    }
    return PX_OK;
}

// --------------------------------------------------------------- autotuner

// Tile rows per problem size: each size class relaxed alone (8 sweeps, one persistent
// launch) for every candidate height, fastest of three timed runs after a warm-up.  Then
// sweeps per launch for the whole batch, by time per sweep: at least 24 sweeps at k =
// 1..8 with the tuned rows, an even number of launches each (so that no candidate pays
// for copying the result back).
int batch_autotune(BatchWork &w, int dtype, const BatchProblem *probs, int nprob, int bc, hipStream_t s,
                   int *best_k, char *err, size_t errlen)
{
    static const int ROWS[] = {4, 6, 8, 12, 16, 20, 24, 29, 32, 38, 40, 48, 64, 96, 128};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        snprintf(err, errlen, "hipEventCreate failed");
        return PX_EHIP;
    }
    int st = PX_OK;
    // time `reps` runs of fn after one warm-up run; returns the fastest in ms (< 0 on error)
    auto fastest = [&](auto &&fn, int reps) -> float {
        if ((st = fn())) return -1.f;
        float best = -1.f;
        for (int r = 0; r < reps; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess) { st = PX_EHIP; return -1.f; }
            if ((st = fn())) return -1.f;
            float ms = 0.f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = PX_EHIP;
                return -1.f;
            }
            if (best < 0.f || ms < best) best = ms;
        }
        return best;
    };
    w.tuned_rows[dtype].clear();
    w.tuned_k[dtype] = 0;
    std::vector<int> sizes;
    for (int p = 0; p < nprob; ++p)
        if (std::find(sizes.begin(), sizes.end(), probs[p].n) == sizes.end()) sizes.push_back(probs[p].n);
    for (int n : sizes) {
        std::vector<BatchProblem> cls;
        for (int p = 0; p < nprob; ++p)
            if (probs[p].n == n) cls.push_back(probs[p]);
        int br = 0;
        float bt = -1.f;
        for (int rows : ROWS) {
            if (rows > std::max(8, n + 2)) break;
            const float ms = fastest([&] {
                return batch_relax(w, dtype, cls.data(), (int)cls.size(), 8, 8, bc, RES_NONE, nullptr, rows, s, err,
                                   errlen);
            }, 3);
            if (st) break;
            if (bt < 0.f || ms < bt) {
                bt = ms;
                br = rows;
            }
        }
        if (st) break;
        w.tuned_rows[dtype].push_back({n, br});
    }
    int bk = 8;
    if (!st) {
        float bt = -1.f;
        for (int k = 1; k <= 8 && !st; ++k) {
            const int sweeps = 2 * k * ((24 + 2 * k - 1) / (2 * k));
            const float ms = fastest([&] {
                return batch_relax(w, dtype, probs, nprob, sweeps, k, bc, RES_NONE, nullptr, 0, s, err, errlen);
            }, 2);
            if (st) break;
            const float per = ms / sweeps;
            if (bt < 0.f || per < bt) {
                bt = per;
                bk = k;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) {
        w.tuned_rows[dtype].clear();
        if (!err[0]) snprintf(err, errlen, "batched autotune: HIP event failure");
        return st;
    }
    w.tuned_k[dtype] = bk;
    if (best_k) *best_k = bk;
    return PX_OK;
}

// ------------------------------------------------------------------ solve

int batch_solve(BatchWork &w, int lowp, const BatchProblem *probs, int nprob, int bc, double rtol,
                int use_l2, long long max_sweeps, int inner, int k, int steps_per_graph, int forced_rows,
                BatchStat *stats, hipStream_t user_stream, char *err, size_t errlen)
{
    const size_t les = (size_t)elem_size(lowp);
    const int L = (inner + k - 1) / k;
    const int krem = inner - (L - 1) * k;
    // ---- layout
    size_t off = 0;
    std::vector<size_t> twin(nprob), da(nprob), db(nprob), rl(nprob);
    std::vector<int> ldl(nprob), row_off(nprob + 1, 0), grow_off(nprob + 1, 0);
    for (int p = 0; p < nprob; ++p) {
        const BatchProblem &q = probs[p];
        ldl[p] = (q.n + 2 + 7) / 8 * 8;
        twin[p] = off;
        off += round256((size_t)(q.n + 2) * q.ld * 8);
        da[p] = off;
        off += round256((size_t)(q.n + 2) * ldl[p] * les);
        db[p] = off;
        off += round256((size_t)(q.n + 2) * ldl[p] * les);
        rl[p] = off;
        off += round256((size_t)q.n * ldl[p] * les);
        row_off[p + 1] = row_off[p] + q.n;
        grow_off[p + 1] = grow_off[p] + q.n + 2;
    }
    const int total_rows = row_off[nprob], total_grow = grow_off[nprob];
    // inner relaxation shapes: k sweeps, and the remainder; two directions each
    struct Shape {
        int k;
        std::vector<KArgs> a[2];
        std::vector<int> toff;
        size_t args_off[2], toff_off;
        int total;
    };
    std::vector<Shape> shapes;
    for (int kk : {k, krem}) {
        if (!shapes.empty() && shapes[0].k == kk) break;
        Shape sh;
        sh.k = kk;
        sh.toff.assign(nprob + 1, 0);
        for (int d = 0; d < 2; ++d) sh.a[d].resize(nprob);
        shapes.push_back(std::move(sh));
    }
    for (auto &sh : shapes) {
        for (int d = 0; d < 2; ++d) {
            sh.args_off[d] = off;
            off += round256(sizeof(KArgs) * nprob);
        }
        sh.toff_off = off;
        off += round256(sizeof(int) * (nprob + 1));
    }
    const size_t refine_off = off;
    off += round256(sizeof(RefineProb) * nprob);
    const size_t rowoff_off = off;
    off += round256(sizeof(int) * (nprob + 1));
    const size_t growoff_off = off;
    off += round256(sizeof(int) * (nprob + 1));
    const size_t state_off = off;  // active, parity (int); steps, sweeps (i64); r0, norms, fnorms (f64)
    off += round256(sizeof(int) * nprob) * 2 + round256(sizeof(long long) * nprob) * 2 +
           round256(sizeof(double) * nprob) * 5;
    const size_t parts = (size_t)std::max(total_rows, 1);
    const size_t pmax_off = off;
    off += round256(parts * 8);
    const size_t psum_off = off;
    off += round256(parts * 8);
    hipError_t e = w.ensure(off);
    if (e != hipSuccess) {
        snprintf(err, errlen, "hipMalloc(%zu) for the batch failed", off);
        return PX_ENOMEM;
    }
    char *base = static_cast<char *>(w.mem);
    size_t so = state_off;
    int *active = dev_ptr<int>(base, so);
    so += round256(sizeof(int) * nprob);
    int *parity = dev_ptr<int>(base, so);
    so += round256(sizeof(int) * nprob);
    long long *steps = dev_ptr<long long>(base, so);
    so += round256(sizeof(long long) * nprob);
    long long *sweeps = dev_ptr<long long>(base, so);
    so += round256(sizeof(long long) * nprob);
    double *r0 = dev_ptr<double>(base, so);
    so += round256(sizeof(double) * nprob);
    double *norms = dev_ptr<double>(base, so);
    so += round256(sizeof(double) * nprob) * 2;
    double *fnorms = dev_ptr<double>(base, so);
    unsigned long long *pmax = dev_ptr<unsigned long long>(base, pmax_off);
    double *psum = dev_ptr<double>(base, psum_off);

    // ---- host-side argument arrays
    std::vector<RefineProb> rp(nprob);
    const int final_is_b = (L % 2 == 1);  // launches alternate a->b, b->a
    for (int p = 0; p < nprob; ++p) {
        const BatchProblem &q = probs[p];
        RefineProb &r = rp[p];
        r.phi[0] = static_cast<double *>(q.phi);
        r.phi[1] = dev_ptr<double>(base, twin[p]);
        r.delta = base + (final_is_b ? db[p] : da[p]);
        r.f = static_cast<const double *>(q.f);
        r.r_low = base + rl[p];
        r.zero = base + da[p];
        r.n = q.n;
        r.ld = q.ld;
        r.ld_f = q.ld_f;
        r.ld_l = ldl[p];
        r.bc = bc;
        r.c = 1.0 / (q.h * q.h);
        for (auto &sh : shapes) {
            const int rows = w.rows_for(lowp, q.n, sh.k, forced_rows);
            sh.a[0][p] = make_kargs(lowp, base + da[p], base + db[p], base + rl[p], q.n, ldl[p], ldl[p], q.h,
                                    q.lambda, bc, sh.k, RES_NONE, rows);
            sh.a[1][p] = make_kargs(lowp, base + db[p], base + da[p], base + rl[p], q.n, ldl[p], ldl[p], q.h,
                                    q.lambda, bc, sh.k, RES_NONE, rows);
            sh.toff[p + 1] = sh.toff[p] + sh.a[0][p].ntiles;
        }
    }
    for (auto &sh : shapes) sh.total = sh.toff[nprob];

    // ---- work stream (capturable) ordered after the caller's stream
    if (!w.stream) {
        hipStream_t ns;
        if ((e = hipStreamCreateWithFlags(&ns, hipStreamNonBlocking)) != hipSuccess) {
            snprintf(err, errlen, "hipStreamCreate: %s", hipGetErrorString(e));
            return PX_EHIP;
        }
        w.stream = ns;
    }
    hipStream_t s = static_cast<hipStream_t>(w.stream);
    hipEvent_t ev;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
        snprintf(err, errlen, "hipEventCreate: %s", hipGetErrorString(e));
        return PX_EHIP;
    }
    e = hipEventRecord(ev, user_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);

    // ---- uploads and state
    std::vector<int> ones(nprob, 1), zeros(nprob, 0);
    std::vector<long long> zl(nprob, 0);
    auto up = [&](void *dst, const void *src, size_t b) {
        if (e == hipSuccess) e = hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, s);
    };
    for (auto &sh : shapes) {
        for (int d = 0; d < 2; ++d) up(base + sh.args_off[d], sh.a[d].data(), sizeof(KArgs) * nprob);
        up(base + sh.toff_off, sh.toff.data(), sizeof(int) * (nprob + 1));
    }
    up(base + refine_off, rp.data(), sizeof(RefineProb) * nprob);
    up(base + rowoff_off, row_off.data(), sizeof(int) * (nprob + 1));
    up(base + growoff_off, grow_off.data(), sizeof(int) * (nprob + 1));
    up(active, ones.data(), sizeof(int) * nprob);
    up(parity, zeros.data(), sizeof(int) * nprob);
    up(steps, zl.data(), sizeof(long long) * nprob);
    up(sweeps, zl.data(), sizeof(long long) * nprob);

    RowArgs ra;
    ra.probs = dev_ptr<const RefineProb>(base, refine_off);
    ra.row_off = dev_ptr<const int>(base, rowoff_off);
    ra.nprob = nprob;
    ra.total_rows = total_rows;
    ra.active = active;
    ra.parity = parity;
    ra.use_delta = 0;
    ra.pmax = pmax;
    ra.psum = psum;
    RowArgs ga = ra;  // over grid rows (n + 2 per problem)
    ga.row_off = dev_ptr<const int>(base, growoff_off);
    ga.total_rows = total_grow;
    CheckArgs ca;
    ca.nprob = nprob;
    ca.active = active;
    ca.parity = parity;
    ca.steps = steps;
    ca.sweeps = sweeps;
    ca.norms = norms;
    ca.fnorms = fnorms;
    ca.r0 = r0;
    ca.use_l2 = use_l2;
    ca.rtol = rtol;
    ca.max_sweeps = max_sweeps;
    ca.inner = 0;
    const dim3 cgrid((nprob + BX - 1) / BX);

    auto refine = [&](const RowArgs &a) {
        if (lowp == F32) hipLaunchKernelGGL(refine_rows_kernel<float>, dim3(total_rows), dim3(BX), 0, s, a);
        else hipLaunchKernelGGL(refine_rows_kernel<bf16>, dim3(total_rows), dim3(BX), 0, s, a);
    };
    auto outer_step = [&]() {
        if (lowp == F32) hipLaunchKernelGGL(zero_rows_kernel<float>, dim3(total_grow), dim3(BX), 0, s, ga);
        else hipLaunchKernelGGL(zero_rows_kernel<bf16>, dim3(total_grow), dim3(BX), 0, s, ga);
        for (int i = 0; i < L; ++i) {
            const Shape &sh = (i == L - 1) ? shapes.back() : shapes[0];
            BatchArgs ba;
            ba.probs = dev_ptr<const KArgs>(base, sh.args_off[i % 2]);
            ba.tile_off = dev_ptr<const int>(base, sh.toff_off);
            ba.active = active;
            ba.nprob = nprob;
            ba.total = sh.total;
            ba.pmax = pmax;
            ba.psum = psum;
            if (hipError_t le = pick_batch(lowp, sh.k, RES_NONE)(ba, s)) return le;
        }
        RowArgs a = ra;
        a.use_delta = 1;
        refine(a);
        hipLaunchKernelGGL(reduce_per_problem_kernel, dim3(nprob), dim3(BX), 0, s, pmax, psum, ra.row_off,
                           (const int *)active, norms);
        CheckArgs c = ca;
        c.inner = inner;
        hipLaunchKernelGGL(check_kernel, cgrid, dim3(BX), 0, s, c);
        return hipGetLastError();
    };

    // ---- norms of f, first residual, first check (not part of the graph)
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fnorm_rows_kernel, dim3(total_rows), dim3(BX), 0, s, ra);
        hipLaunchKernelGGL(reduce_per_problem_kernel, dim3(nprob), dim3(BX), 0, s, pmax, psum, ra.row_off,
                           (const int *)nullptr, fnorms);
        refine(ra);
        hipLaunchKernelGGL(reduce_per_problem_kernel, dim3(nprob), dim3(BX), 0, s, pmax, psum, ra.row_off,
                           (const int *)active, norms);
        hipLaunchKernelGGL(check_kernel, cgrid, dim3(BX), 0, s, ca);
        e = hipGetLastError();
    }
    // ---- capture `steps_per_graph` outer steps once
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t ce = hipSuccess;
        for (int i = 0; i < steps_per_graph && ce == hipSuccess; ++i) ce = outer_step();
        e = hipStreamEndCapture(s, &graph);
        if (e == hipSuccess) e = ce;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    // ---- replay until no problem is running
    std::vector<int> act(nprob, 1);
    while (e == hipSuccess) {
        e = hipMemcpyAsync(act.data(), active, sizeof(int) * nprob, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) break;
        if (std::none_of(act.begin(), act.end(), [](int v) { return v == ST_RUN; })) break;
        e = hipGraphLaunch(exec, s);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(copyback_rows_kernel, dim3(total_grow), dim3(BX), 0, s, ga);
        e = hipGetLastError();
    }
    std::vector<long long> hs(nprob), hw(nprob);
    std::vector<double> hn(2 * nprob), hf(2 * nprob);
    if (e == hipSuccess) e = hipMemcpyAsync(hs.data(), steps, sizeof(long long) * nprob, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hw.data(), sweeps, sizeof(long long) * nprob, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hn.data(), norms, sizeof(double) * 2 * nprob, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hf.data(), fnorms, sizeof(double) * 2 * nprob, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) {
        snprintf(err, errlen, "batched solve: %s", hipGetErrorString(e));
        return PX_EHIP;
    }
    int status = PX_OK;
    for (int p = 0; p < nprob; ++p) {
        BatchStat &b = stats[p];
        b.state = act[p];
        b.steps = hs[p];
        b.sweeps = hw[p];
        b.res_max = hn[2 * p];
        b.res_l2 = std::sqrt(hn[2 * p + 1]);
        b.rel_res_max = hf[2 * p] > 0 ? hn[2 * p] / hf[2 * p] : hn[2 * p];
        b.rel_res_l2 = hf[2 * p + 1] > 0 ? std::sqrt(hn[2 * p + 1] / hf[2 * p + 1]) : b.res_l2;
        if (status == PX_OK && act[p] != ST_DONE)
            status = act[p] == ST_BUDGET ? PX_ENOTCONV : act[p] == ST_NONFINITE ? PX_ENONFINITE : PX_EDIVERGED;
    }
    if (status != PX_OK) snprintf(err, errlen, "not every problem of the batch converged");
    return status;
}

}  // namespace px
