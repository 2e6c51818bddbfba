// px_internal.h -- shared internals of the gfx950 HIP library (not part of the ABI).
//
// Element-type traits, the bfloat16 rounding used on every BF16 store, the
// launcher descriptors the host API fills in, and the launcher prototypes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

struct px_net;

namespace px {

enum Dtype { F64 = 0, F32 = 1, BF16 = 2 };
enum Bc { DIRICHLET0 = 0, GHOST_FIXED = 1, PERIODIC = 2 };
enum ResMode { RES_NONE = 0, RES_LAGGED = 1, RES_FINAL = 2 };

struct bf16 {
    uint16_t bits;
};

// Round-to-nearest-even of a binary32 to bfloat16: gfx950's v_cvt_pk_bf16_f32, which
// rounds ties to even, keeps denormals, and turns a NaN into a quiet NaN with its sign and
// upper payload bits ((bits >> 16) | 0x40) -- checked on the device against the integer
// formulation over every upper half-word with tie, near-tie and zero lower half-words.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Storage traits: A is the arithmetic type, load/store convert, round() gives the
// arithmetic value of what a store followed by a load would produce.
template <typename T> struct Elem;
template <> struct Elem<double> {
    using A = double;
    static constexpr int code = F64;
    __device__ static A load(double x) { return x; }
    __device__ static double store(A x) { return x; }
    __device__ static A round(A x) { return x; }
};
template <> struct Elem<float> {
    using A = float;
    static constexpr int code = F32;
    __device__ static A load(float x) { return x; }
    __device__ static float store(A x) { return x; }
    __device__ static A round(A x) { return x; }
};
template <> struct Elem<bf16> {
    using A = float;
    static constexpr int code = BF16;
    __device__ static A load(bf16 x) { return bf16_to_f32(x.bits); }
    __device__ static bf16 store(A x) { return bf16{f32_to_bf16_rne(x)}; }
    __device__ static A round(A x) { return bf16_to_f32(f32_to_bf16_rne(x)); }
};

// N - 4C rounded once.  Scaling by 4 is exact while 4|C| stays finite (|C| up to a quarter of
// the largest finite value), so there the fused form rounds the same exact difference as
// forming 4C and then subtracting -- the same bits -- in one instruction instead of two.
__device__ __forceinline__ double sub4(double N, double C) { return __builtin_fma(-4.0, C, N); }
__device__ __forceinline__ float sub4(float N, float C) { return __builtin_fmaf(-4.0f, C, N); }

inline int elem_size(int dtype) { return dtype == F64 ? 8 : dtype == F32 ? 4 : 2; }

// Per-wave (or per-block) partial norms: max|r| as the bit pattern of a
// non-negative double (integer order == value order, NaN above +Inf) and the
// sum of r^2.
struct Partials {
    unsigned long long *max_bits;
    double *sum;
};

struct RelaxLaunch {
    const void *in;
    void *out;
    const void *f;
    int n, ld, ld_f;
    double c, w, lam;  // 1/h^2, lambda/h^2, lambda (FP64; rounded once for FP32/BF16)
    int bc;
    int sweeps;        // sweeps in this launch (1..8)
    int resmode;       // RES_NONE / RES_LAGGED / RES_FINAL for this launch
    int rows;          // rows per wave tile
    Partials part;     // needs >= relax_num_waves() entries when resmode != RES_NONE
};

// Number of wave tiles (== partial slots) a launch with these settings uses.
int relax_num_waves(int dtype, int n, int sweeps, int resmode, int rows);
// Default rows per tile for a given problem and sweeps per launch.
int relax_default_rows(int dtype, int n, int sweeps);
hipError_t relax_launch(int dtype, const RelaxLaunch &a, hipStream_t s);

// Fixed-order reduction of `count` partials into norms[0] = max, norms[1] = sum.
hipError_t reduce_partials(Partials p, int count, double *norms, hipStream_t s);
int pointwise_num_blocks(int n);

hipError_t stencil_launch(int dtype, const void *phi, int n, int ld, void *out, int ld_out,
                          const double taps[9], double scale, int bc, hipStream_t s);
hipError_t residual_launch(int dtype, const void *phi, int n, int ld, const void *f, int ld_f,
                           double c, int bc, void *r, int ld_r, Partials part, hipStream_t s);
hipError_t jacobi_launch(int dtype, void *phi, int n, int ld, const void *sv, int ld_s,
                         const void *f, int ld_f, double w, double lam, hipStream_t s);
hipError_t copy_grid_launch(int dtype, const void *in, void *out, int n, int ld, hipStream_t s);

// Mixed-precision refinement pieces (FP64 outer step).
// phi_out = phi_in + delta (interior; delta of dtype lowp with leading dimension
// ld_d, may be NULL for 0), r = f - L phi_out: FP64 partial norms, and r rounded
// to lowp into r_low.
hipError_t refine_launch(int lowp, const double *phi_in, const void *delta, int ld_d, double *phi_out,
                         int n, int ld, const double *f, int ld_f, double c, int bc,
                         void *r_low, int ld_r, Partials part, hipStream_t s);
hipError_t zero_grid_launch(int dtype, void *p, int n, int ld, hipStream_t s);

// ---- batches of independent problems (batched.hip)
struct BatchProblem {
    void *phi;        // (n+2) x ld, in place
    const void *f;    // n x ld_f
    int n, ld, ld_f;
    double h, lambda;
};
struct BatchStat {
    int state;        // 0 converged, -1 sweep budget, -2 non-finite, -3 diverged
    long long steps, sweeps;
    double res_max, res_l2, rel_res_max, rel_res_l2;
};
// Device memory, work stream and graph of batched calls, owned by a context.
struct BatchWork {
    void *mem = nullptr;
    size_t bytes = 0;
    void *stream = nullptr;
    void *graph_exec = nullptr;
    // autotuned per element type: sweeps per launch (0 = not tuned) and tile rows per
    // problem size n (sizes not listed use the built-in heuristic)
    int tuned_k[3] = {0, 0, 0};
    std::vector<std::pair<int, int>> tuned_rows[3];
    int rows_for(int dtype, int n, int k, int forced) const;
    ~BatchWork();
    hipError_t ensure(size_t need);
};
int batch_relax(BatchWork &w, int dtype, const BatchProblem *probs, int nprob, int nsweeps, int k, int bc,
                int resmode, double *norms, int forced_rows, hipStream_t s, char *err, size_t errlen);
// Boxes of one domain (px_relax_boxes): nbx x nby boxes of equal n in row-major order, in
// place; every `exchange` sweeps the ghost rings are refreshed from the neighbouring boxes
// (domain edges per bc), then every box relaxes `exchange` sweeps with fixed ghosts.
int batch_relax_boxes(BatchWork &w, int dtype, const BatchProblem *probs, int nbx, int nby, int nsweeps, int exchange,
                      int bc, int forced_rows, hipStream_t s, char *err, size_t errlen);
// Autotuner of batched relaxation (see px_autotune_batched); relaxes the problems in place.
int batch_autotune(BatchWork &w, int dtype, const BatchProblem *probs, int nprob, int bc, hipStream_t s,
                   int *best_k, char *err, size_t errlen);
int batch_solve(BatchWork &w, int lowp, const BatchProblem *probs, int nprob, int bc, double rtol,
                int use_l2, long long max_sweeps, int inner, int k, int steps_per_graph, int forced_rows,
                BatchStat *stats, hipStream_t user_stream, char *err, size_t errlen);

// ---- learned correction (net.hip)
// Records the message of a failing ABI call (px_last_error) and returns code.
int set_error(int code, const char *fmt, ...);
// y (FP32, rows of ld_y) = N(r * scale) for one n x n image r (FP64, rows of ld_r).
hipError_t net_infer(px_net *net, const double *r, int ld_r, int n, double scale, float *y, int ld_y,
                     hipStream_t s);
int net_device(const px_net *net);
// Training pair pieces: sums[0] = sum S(phi)^2, sums[1] = sum e^2 (loss MSE) or sum e K e
// (loss ENERGY), e = -phi; then x = -S(phi) / rms, t = e / rms.  part: >= pair_num_blocks(n)
// double2 slots.
int pair_num_blocks(int n);
hipError_t pair_launch(const double *phi, int n, int ld, int loss, float *x, float *t, double *part,
                       double *sums, hipStream_t s);
// Correction step of the learned refinement: the five sums {<r,r>, <d,r>, <r,Sr>, <r,Sd>,
// <d,Sd>} (S with odd reflection; d compact n x ld_d, FP32 or FP64) into dots (5 doubles),
// then phi += a r + b d with the energy-optimal (a, b) for `mode` (0: r, 1: d, 2: both);
// coef (may be NULL) receives (a, b).  part: >= 8 * pair_num_blocks(n) doubles.
hipError_t correction_launch(int ddtype, const void *d, int ld_d, const double *r, int ld_r, double *phi, int n,
                             int ld, double c, int mode, double *part, double *dots, double *coef, hipStream_t s);

}  // namespace px
