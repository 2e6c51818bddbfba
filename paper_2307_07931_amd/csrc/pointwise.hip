// pointwise.hip -- the unfused building blocks and the reductions.
//
//   stencil_kernel   out = scale * S(phi) for general 3x3 taps (Eq. 1), the
//                    standalone stencil of the unfused (Proto-shaped) sweep;
//   residual_kernel  r = f - (1/h^2) S(phi) plus per-block partial norms
//                    (the OL max-norm expression; also sum r^2);
//   jacobi_kernel    the pointwise update phi = (phi + w s) - lambda f, in
//                    place (Proto's forallInPlace step);
//   refine_kernel    FP64 outer step of mixed-precision refinement:
//                    phi_out = phi_in + delta, r = f - L phi_out, r rounded
//                    to FP32 (or FP32 then BF16) for the inner solve;
//   reduce_kernel    fixed-order reduction of partial norms.
// Each thread handles one cell; blocks are 256 columns of one row.  These
// kernels are bandwidth-bound streams; neighbour reuse comes from the caches.
#include "px_internal.h"

namespace px {
namespace {

constexpr int BX = 256;

// Fixed-order block reduction of (max bits, sum) -> thread 0.
__device__ __forceinline__ void block_reduce(unsigned long long &mx, double &sm)
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

__device__ __forceinline__ unsigned long long abs_bits(double x)
{
    return (unsigned long long)__double_as_longlong(fabs(x));
}

// Neighbour fetch of phi at (i, j) honouring the boundary mode; (ci, cj) is the
// interior cell the neighbour belongs to, C its value.
// Boundary modes of these per-cell kernels: DIRICHLET0 (odd reflection), GHOST_FIXED (the
// ghost as stored), PERIODIC (the interior cell n cells away).
__device__ __forceinline__ int wrap_index(int i, int n) { return i == 0 ? n : (i == n + 1 ? 1 : i); }

template <typename T>
__device__ __forceinline__ typename Elem<T>::A nb(const T *__restrict__ phi, int ld, int n, int i,
                                                  int j, typename Elem<T>::A C, int bc)
{
    if (bc == DIRICHLET0 && (i == 0 || i == n + 1 || j == 0 || j == n + 1)) return -C;
    if (bc == PERIODIC) {
        i = wrap_index(i, n);
        j = wrap_index(j, n);
    }
    return Elem<T>::load(phi[(size_t)i * ld + j]);
}

// Corner ghost under DIRICHLET0 (general taps only): +(diagonal interior).
template <typename T>
__device__ __forceinline__ typename Elem<T>::A at_reflected(const T *__restrict__ phi, int ld,
                                                            int n, int i, int j, int bc)
{
    using A = typename Elem<T>::A;
    if (bc == PERIODIC) return Elem<T>::load(phi[(size_t)wrap_index(i, n) * ld + wrap_index(j, n)]);
    if (bc != DIRICHLET0) return Elem<T>::load(phi[(size_t)i * ld + j]);
    int ii = i, jj = j;
    A sgn = 1;
    if (ii == 0) { ii = 1; sgn = -sgn; }
    if (ii == n + 1) { ii = n; sgn = -sgn; }
    if (jj == 0) { jj = 1; sgn = -sgn; }
    if (jj == n + 1) { jj = n; sgn = -sgn; }
    const A v = Elem<T>::load(phi[(size_t)ii * ld + jj]);
    return sgn < 0 ? -v : v;
}

template <typename T>
__device__ __forceinline__ typename Elem<T>::A lap5(const T *__restrict__ phi, int ld, int n, int i,
                                                    int j, int bc, typename Elem<T>::A &C)
{
    using A = typename Elem<T>::A;
    C = Elem<T>::load(phi[(size_t)i * ld + j]);
    const A N = nb<T>(phi, ld, n, i - 1, j, C, bc);
    const A W = nb<T>(phi, ld, n, i, j - 1, C, bc);
    const A E = nb<T>(phi, ld, n, i, j + 1, C, bc);
    const A S = nb<T>(phi, ld, n, i + 1, j, C, bc);
    return (((N - (A)4 * C) + W) + E) + S;
}

struct Taps {
    double t[9];
};

template <typename T, bool LAP>
__global__ __launch_bounds__(BX) void stencil_kernel(const T *__restrict__ phi, int n, int ld,
                                                     T *__restrict__ out, int ld_out, Taps taps,
                                                     double scale, int apply_scale, int bc)
{
    using A = typename Elem<T>::A;
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y + 1;
    if (j > n) return;
    A acc;
    if (LAP) {
        A C;
        acc = lap5<T>(phi, ld, n, i, j, bc, C);
    } else {
        // visiting order (-1,0), (0,0), (0,-1), (0,1), (1,0), corners; zero taps skipped
        const int di[9] = {-1, 0, 0, 0, 1, -1, -1, 1, 1};
        const int dj[9] = {0, 0, -1, 1, 0, -1, 1, -1, 1};
        bool first = true;
        acc = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const A tap = (A)taps.t[(di[k] + 1) * 3 + (dj[k] + 1)];
            if (tap == (A)0) continue;
            const A term = tap * at_reflected<T>(phi, ld, n, i + di[k], j + dj[k], bc);
            acc = first ? term : acc + term;
            first = false;
        }
    }
    if (apply_scale) acc = (A)scale * acc;
    out[(size_t)(i - 1) * ld_out + (j - 1)] = Elem<T>::store(acc);
}

template <typename T>
__global__ __launch_bounds__(BX) void residual_kernel(const T *__restrict__ phi, int n, int ld,
                                                      const T *__restrict__ f, int ld_f, double c,
                                                      int bc, T *__restrict__ r, int ld_r,
                                                      unsigned long long *pmax, double *psum)
{
    using A = typename Elem<T>::A;
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y + 1;
    unsigned long long mx = 0;
    double sm = 0.0;
    if (j <= n) {
        A C;
        const A s = lap5<T>(phi, ld, n, i, j, bc, C);
        const A rr = Elem<T>::load(f[(size_t)(i - 1) * ld_f + (j - 1)]) - (A)c * s;
        if (r) r[(size_t)(i - 1) * ld_r + (j - 1)] = Elem<T>::store(rr);
        const double rd = (double)rr;
        mx = abs_bits(rd);
        sm = rd * rd;
    }
    block_reduce(mx, sm);
    if (threadIdx.x == 0 && pmax) {
        const int blk = blockIdx.y * gridDim.x + blockIdx.x;
        pmax[blk] = mx;
        psum[blk] = sm;
    }
}

template <typename T>
__global__ __launch_bounds__(BX) void jacobi_kernel(T *__restrict__ phi, int n, int ld,
                                                    const T *__restrict__ sv, int ld_s,
                                                    const T *__restrict__ f, int ld_f, double w,
                                                    double lam)
{
    using A = typename Elem<T>::A;
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y + 1;
    if (j > n) return;
    const size_t q = (size_t)i * ld + j;
    const A p = Elem<T>::load(phi[q]);
    const A s = Elem<T>::load(sv[(size_t)(i - 1) * ld_s + (j - 1)]);
    const A rho = Elem<T>::load(f[(size_t)(i - 1) * ld_f + (j - 1)]);
    phi[q] = Elem<T>::store((p + (A)w * s) - (A)lam * rho);
}

// Copy of every non-corner cell of an (n+2) x ld grid.
template <typename T>
__global__ __launch_bounds__(BX) void copy_grid_kernel(const T *__restrict__ in, T *__restrict__ out,
                                                       int n, int ld)
{
    const int j = blockIdx.x * BX + threadIdx.x;
    const int i = blockIdx.y;
    if (j > n + 1) return;
    if ((i == 0 || i == n + 1) && (j == 0 || j == n + 1)) return;
    const size_t q = (size_t)i * ld + j;
    out[q] = in[q];
}

template <typename T>
__global__ __launch_bounds__(BX) void zero_grid_kernel(T *__restrict__ p, int n, int ld)
{
    const int j = blockIdx.x * BX + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= ld) return;
    p[(size_t)i * ld + j] = T{};
}

// FP64 outer refinement step around a low-precision inner solve.
template <typename L>
__global__ __launch_bounds__(BX) void refine_kernel(const double *__restrict__ phi_in,
                                                    const L *__restrict__ delta, int ld_d,
                                                    double *__restrict__ phi_out, int n, int ld,
                                                    const double *__restrict__ f, int ld_f,
                                                    double c, int bc, L *__restrict__ r_low,
                                                    int ld_r, unsigned long long *pmax,
                                                    double *psum)
{
    const int j = blockIdx.x * BX + threadIdx.x + 1;
    const int i = blockIdx.y + 1;
    unsigned long long mx = 0;
    double sm = 0.0;
    const bool dir = (bc == DIRICHLET0);
    if (j <= n) {
        // updated value of a cell: interior cells add delta, ghosts do not change
        auto upd = [&](int ii, int jj) -> double {
            double v = phi_in[(size_t)ii * ld + jj];
            if (delta && ii >= 1 && ii <= n && jj >= 1 && jj <= n)
                v = v + (double)Elem<L>::load(delta[(size_t)ii * ld_d + jj]);
            return v;
        };
        const double C = upd(i, j);
        const double N = (dir && i == 1) ? -C : upd(i - 1, j);
        const double W = (dir && j == 1) ? -C : upd(i, j - 1);
        const double E = (dir && j == n) ? -C : upd(i, j + 1);
        const double S = (dir && i == n) ? -C : upd(i + 1, j);
        const double s = (((N - 4.0 * C) + W) + E) + S;
        const double rr = f[(size_t)(i - 1) * ld_f + (j - 1)] - c * s;
        const size_t q = (size_t)i * ld + j;
        phi_out[q] = C;
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
        if (r_low) r_low[(size_t)(i - 1) * ld_r + (j - 1)] = Elem<L>::store((float)rr);
        mx = abs_bits(rr);
        sm = rr * rr;
    }
    block_reduce(mx, sm);
    if (threadIdx.x == 0) {
        const int blk = blockIdx.y * gridDim.x + blockIdx.x;
        pmax[blk] = mx;
        psum[blk] = sm;
    }
}

__global__ __launch_bounds__(1024) void reduce_kernel(const unsigned long long *__restrict__ pmax,
                                                      const double *__restrict__ psum, int count,
                                                      double *__restrict__ norms)
{
    __shared__ unsigned long long smx[1024];
    __shared__ double ssm[1024];
    unsigned long long mx = 0;
    double sm = 0.0;
    for (int k = threadIdx.x; k < count; k += 1024) {
        mx = pmax[k] > mx ? pmax[k] : mx;
        sm = sm + psum[k];
    }
    smx[threadIdx.x] = mx;
    ssm[threadIdx.x] = sm;
    __syncthreads();
    for (int half = 512; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) {
            const unsigned long long o = smx[threadIdx.x + half];
            smx[threadIdx.x] = o > smx[threadIdx.x] ? o : smx[threadIdx.x];
            ssm[threadIdx.x] = ssm[threadIdx.x] + ssm[threadIdx.x + half];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        norms[0] = __longlong_as_double((long long)smx[0]);
        norms[1] = ssm[0];
    }
}

inline dim3 interior_grid(int n) { return dim3((n + BX - 1) / BX, n); }
inline dim3 full_grid(int n, int cols) { return dim3((cols + BX - 1) / BX, n + 2); }

}  // namespace

int pointwise_num_blocks(int n) { return ((n + BX - 1) / BX) * n; }

hipError_t reduce_partials(Partials p, int count, double *norms, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, s, p.max_bits, p.sum, count, norms);
    return hipGetLastError();
}

hipError_t stencil_launch(int dtype, const void *phi, int n, int ld, void *out, int ld_out,
                          const double taps[9], double scale, int bc, hipStream_t s)
{
    Taps tp;
    bool lap = true;
    static const double L5[9] = {0, 1, 0, 1, -4, 1, 0, 1, 0};
    for (int k = 0; k < 9; ++k) {
        tp.t[k] = taps[k];
        if (taps[k] != L5[k]) lap = false;
    }
    const int sc = (scale != 1.0) ? 1 : 0;
    const dim3 g = interior_grid(n);
#define PX_STENCIL(T)                                                                             \
    if (lap)                                                                                      \
        hipLaunchKernelGGL((stencil_kernel<T, true>), g, dim3(BX), 0, s, (const T *)phi, n, ld,   \
                           (T *)out, ld_out, tp, scale, sc, bc);                                  \
    else                                                                                          \
        hipLaunchKernelGGL((stencil_kernel<T, false>), g, dim3(BX), 0, s, (const T *)phi, n, ld,  \
                           (T *)out, ld_out, tp, scale, sc, bc);
    switch (dtype) {
    case F64: PX_STENCIL(double) break;
    case F32: PX_STENCIL(float) break;
    case BF16: PX_STENCIL(bf16) break;
    default: return hipErrorInvalidValue;
    }
#undef PX_STENCIL
    return hipGetLastError();
}

hipError_t residual_launch(int dtype, const void *phi, int n, int ld, const void *f, int ld_f,
                           double c, int bc, void *r, int ld_r, Partials part, hipStream_t s)
{
    const dim3 g = interior_grid(n);
#define PX_RES(T)                                                                                 \
    hipLaunchKernelGGL((residual_kernel<T>), g, dim3(BX), 0, s, (const T *)phi, n, ld,            \
                       (const T *)f, ld_f, c, bc, (T *)r, ld_r, part.max_bits, part.sum);
    switch (dtype) {
    case F64: PX_RES(double) break;
    case F32: PX_RES(float) break;
    case BF16: PX_RES(bf16) break;
    default: return hipErrorInvalidValue;
    }
#undef PX_RES
    return hipGetLastError();
}

hipError_t jacobi_launch(int dtype, void *phi, int n, int ld, const void *sv, int ld_s,
                         const void *f, int ld_f, double w, double lam, hipStream_t s)
{
    const dim3 g = interior_grid(n);
#define PX_JAC(T)                                                                                 \
    hipLaunchKernelGGL((jacobi_kernel<T>), g, dim3(BX), 0, s, (T *)phi, n, ld, (const T *)sv,     \
                       ld_s, (const T *)f, ld_f, w, lam);
    switch (dtype) {
    case F64: PX_JAC(double) break;
    case F32: PX_JAC(float) break;
    case BF16: PX_JAC(bf16) break;
    default: return hipErrorInvalidValue;
    }
#undef PX_JAC
    return hipGetLastError();
}

hipError_t copy_grid_launch(int dtype, const void *in, void *out, int n, int ld, hipStream_t s)
{
    const dim3 g = full_grid(n, n + 2);
#define PX_COPY(T)                                                                                \
    hipLaunchKernelGGL((copy_grid_kernel<T>), g, dim3(BX), 0, s, (const T *)in, (T *)out, n, ld);
    switch (dtype) {
    case F64: PX_COPY(double) break;
    case F32: PX_COPY(float) break;
    case BF16: PX_COPY(bf16) break;
    default: return hipErrorInvalidValue;
    }
#undef PX_COPY
    return hipGetLastError();
}

hipError_t zero_grid_launch(int dtype, void *p, int n, int ld, hipStream_t s)
{
    const dim3 g = full_grid(n, ld);
    switch (dtype) {
    case F64: hipLaunchKernelGGL((zero_grid_kernel<double>), g, dim3(BX), 0, s, (double *)p, n, ld); break;
    case F32: hipLaunchKernelGGL((zero_grid_kernel<float>), g, dim3(BX), 0, s, (float *)p, n, ld); break;
    case BF16: hipLaunchKernelGGL((zero_grid_kernel<bf16>), g, dim3(BX), 0, s, (bf16 *)p, n, ld); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t refine_launch(int lowp, const double *phi_in, const void *delta, int ld_d, double *phi_out,
                         int n, int ld, const double *f, int ld_f, double c, int bc, void *r_low,
                         int ld_r, Partials part, hipStream_t s)
{
    const dim3 g = interior_grid(n);
    if (lowp == F32)
        hipLaunchKernelGGL((refine_kernel<float>), g, dim3(BX), 0, s, phi_in, (const float *)delta,
                           ld_d, phi_out, n, ld, f, ld_f, c, bc, (float *)r_low, ld_r, part.max_bits,
                           part.sum);
    else if (lowp == BF16)
        hipLaunchKernelGGL((refine_kernel<bf16>), g, dim3(BX), 0, s, phi_in, (const bf16 *)delta,
                           ld_d, phi_out, n, ld, f, ld_f, c, bc, (bf16 *)r_low, ld_r, part.max_bits,
                           part.sum);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace px
