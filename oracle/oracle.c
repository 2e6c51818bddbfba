/*
 * oracle.c -- plain, slow CPU reference for the fused Poisson relaxation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the HIP library.
 *
 * What it computes (ProtoX paper, Section IV "2D Poisson equation" and
 * "Algorithm"):
 *   - the 2D Poisson problem  Laplace(phi) = rho  on the unit square (Eq. 2),
 *   - discretised with the 5-point stencil S, a special case of the generic
 *     constant-coefficient stencil  S(x)_i = sum_j alpha_j x_{i+j}  (Eq. 1),
 *     with taps [0,1,0; 1,-4,1; 0,1,0] (the filter t of the OL expression),
 *   - one Jacobi step  phi^n = phi^{n-1} + lambda (S(phi^{n-1})/h^2 - rho)
 *     (Eq. 3), written in the OL form Jacobi = (1, w, -lambda) (x) I with
 *     w = lambda/h^2 acting on [phi; S phi; rho],
 *   - the max-norm  || (0, 1/h^2, -1) (x) I [phi; S phi; rho] ||_inf  of the
 *     OL expression for the norm, i.e. the residual of the iterate that the
 *     sweep READS (the OL places Jacobi and the norm side by side on the same
 *     input).
 *
 * The sweep is evaluated exactly as the three-step algorithm states it, one
 * full pass per step and a separate temporary for S(phi): (1) apply the
 * Laplacian, (2) the Jacobi update into a separate output array, (3) the
 * max-norm.  No fusion, tiling or reordering.
 *
 * Readings (the paper is silent or ambiguous on these):
 *   - association: the stencil sum is ((((N - 4C) + W) + E) + S) and the
 *     update is ((phi + w*s) - lambda*rho), the order the generated fused
 *     code in the paper's CPU figure uses; no fused multiply-add (compile
 *     with -ffp-contract=off);
 *   - boundary: homogeneous Dirichlet at the cell faces of a cell-centred
 *     grid (h = 1/n), realised as odd reflection: ghost = -(adjacent
 *     interior), refreshed before every sweep; corner ghosts = +(diagonal
 *     interior) (reflection in both directions).  The alternative
 *     GHOST_FIXED mode reads the ghost ring as given and never changes it
 *     (the literal behaviour of the paper's generated code, which reads
 *     ghost cells and never writes them).  PERIODIC (Proto's own boundary,
 *     Section II) wraps the grid into a torus: each ghost is a copy of the
 *     interior cell n cells away (corners included), refreshed before every
 *     sweep and written with the output;
 *   - residual vector:  r = rho - (1/h^2) s.  The paper's norm takes
 *     |(1/h^2) s - rho|, which is the same number bit for bit;
 *   - the max is NaN-propagating (a NaN residual makes the norm NaN);
 *   - also reported: sum of r^2 (for the L2 norm), accumulated in FP64 in
 *     plain row-major order.
 *
 * Layout: phi is (n+2) rows x ld doubles, row-major, interior at rows and
 * columns 1..n, ghost ring around it.  rho (called f here) is n rows x ld_f,
 * compact, f[(i-1)*ld_f + (j-1)] belongs to phi cell (i, j).
 *
 * Precision variants:
 *   ox_*_f64   FP64 storage and arithmetic (the oracle proper),
 *   ox_*_f32   FP32 storage and arithmetic, constants rounded once from FP64,
 *   ox_*_bf16  bfloat16 storage (round-to-nearest-even on every store),
 *              FP32 arithmetic.
 * All three follow the same steps; only the storage type changes.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the row loops (OpenMP).  Every parallel loop below writes disjoint
 * rows and reduces nothing, so results are identical for any thread count; the
 * one reduction of a sweep (the sum of squares in the norm pass) stays a single
 * sequential loop in row-major order. */
static int ox_threads = 1;
void ox_set_threads(int t) { ox_threads = t > 0 ? t : 1; }
int ox_get_threads(void) { return ox_threads; }
int ox_max_threads(void) { return omp_get_num_procs(); }
#define OX_ROWS _Pragma("omp parallel for schedule(static) num_threads(ox_threads)")

enum { OX_BC_DIRICHLET0 = 0, OX_BC_GHOST_FIXED = 1, OX_BC_PERIODIC = 2 };
enum { OX_RES_NONE = 0, OX_RES_LAGGED = 1, OX_RES_FINAL = 2 };

/* ------------------------------------------------------------------ */
/* bfloat16 storage: top 16 bits of an IEEE binary32, rounded to nearest,
 * ties to even; NaN stays NaN (quiet).                                  */
/* ------------------------------------------------------------------ */
uint16_t ox_f32_to_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu) != 0)
        return (uint16_t)((u >> 16) | 0x0040u); /* quiet NaN */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

float ox_bf16_to_f32(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float x;
    memcpy(&x, &u, 4);
    return x;
}

/* NaN-propagating maximum of non-negative magnitudes. */
static double nanmax_d(double a, double b)
{
    if (isnan(a)) return a;
    if (isnan(b)) return b;
    return (b > a) ? b : a;
}

/* Visiting order of the nine taps of a 3x3 stencil, as (row, col) offsets.
 * For the 5-point Laplacian this is exactly the order N, C, W, E, S of the
 * paper's generated code; zero taps are skipped entirely. */
static const int TAP_ORDER[9][2] = {
    {-1, 0}, {0, 0}, {0, -1}, {0, 1}, {1, 0},
    {-1, -1}, {-1, 1}, {1, -1}, {1, 1}};

/* ================================================================== */
/* Type-generic body, instantiated for (storage, arithmetic) pairs.     */
/* LOAD(x) turns a stored value into the arithmetic type, STORE(v)      */
/* rounds an arithmetic value into storage.                            */
/* ================================================================== */
#define OX_DEFINE(SUF, ST, AT, LOAD, STORE)                                          \
                                                                                     \
/* Step 0: a working copy of phi with the ghost ring refreshed per side.          \
 * bcs[0..3] = mode of the north (row 0), south (row n+1), west (column 0) and    \
 * east (column n+1) ghost layers.  Corners are reflected only where both        \
 * adjacent sides reflect. */                                                     \
static void ghosted_fill_##SUF(const ST *phi, int n, int ld, const int bcs[4], AT *w)  \
{                                                                                    \
    int m = n + 2;                                                                   \
    OX_ROWS                                                                          \
    for (int i = 0; i < m; ++i)                                                      \
        for (int j = 0; j < m; ++j)                                                  \
            w[(size_t)i * m + j] = LOAD(phi[(size_t)i * ld + j]);                    \
    for (int k = 1; k <= n; ++k) {                                                   \
        if (bcs[0] == OX_BC_DIRICHLET0) w[(size_t)0 * m + k] = -w[(size_t)1 * m + k];\
        if (bcs[1] == OX_BC_DIRICHLET0)                                              \
            w[(size_t)(n + 1) * m + k] = -w[(size_t)n * m + k];                      \
        if (bcs[2] == OX_BC_DIRICHLET0) w[(size_t)k * m + 0] = -w[(size_t)k * m + 1];\
        if (bcs[3] == OX_BC_DIRICHLET0)                                              \
            w[(size_t)k * m + (n + 1)] = -w[(size_t)k * m + n];                      \
    }                                                                                \
    for (int k = 1; k <= n; ++k) {                                                   \
        if (bcs[0] == OX_BC_PERIODIC) w[(size_t)0 * m + k] = w[(size_t)n * m + k];   \
        if (bcs[1] == OX_BC_PERIODIC) w[(size_t)(n + 1) * m + k] = w[(size_t)1 * m + k]; \
        if (bcs[2] == OX_BC_PERIODIC) w[(size_t)k * m + 0] = w[(size_t)k * m + n];   \
        if (bcs[3] == OX_BC_PERIODIC) w[(size_t)k * m + (n + 1)] = w[(size_t)k * m + 1]; \
    }                                                                                \
    if (bcs[0] == OX_BC_PERIODIC && bcs[2] == OX_BC_PERIODIC) {                      \
        w[0] = w[(size_t)n * m + n];                                                 \
        w[n + 1] = w[(size_t)n * m + 1];                                             \
        w[(size_t)(n + 1) * m + 0] = w[(size_t)1 * m + n];                           \
        w[(size_t)(n + 1) * m + n + 1] = w[(size_t)1 * m + 1];                       \
    }                                                                                \
    if (bcs[0] == OX_BC_DIRICHLET0 && bcs[2] == OX_BC_DIRICHLET0)                    \
        w[0] = w[(size_t)1 * m + 1];                                                 \
    if (bcs[0] == OX_BC_DIRICHLET0 && bcs[3] == OX_BC_DIRICHLET0)                    \
        w[n + 1] = w[(size_t)1 * m + n];                                             \
    if (bcs[1] == OX_BC_DIRICHLET0 && bcs[2] == OX_BC_DIRICHLET0)                    \
        w[(size_t)(n + 1) * m + 0] = w[(size_t)n * m + 1];                           \
    if (bcs[1] == OX_BC_DIRICHLET0 && bcs[3] == OX_BC_DIRICHLET0)                    \
        w[(size_t)(n + 1) * m + n + 1] = w[(size_t)n * m + n];                       \
}                                                                                    \
static AT *ghosted_copy_##SUF(const ST *phi, int n, int ld, const int bcs[4])       \
{                                                                                    \
    AT *w = (AT *)malloc(sizeof(AT) * (size_t)(n + 2) * (n + 2));                    \
    ghosted_fill_##SUF(phi, n, ld, bcs, w);                                          \
    return w;                                                                        \
}                                                                                    \
                                                                                     \
/* Step 1 (Eq. 1): temp(i,j) = sum over nonzero taps of tap * phi(i+a, j+b), in the  \
 * fixed visiting order, for the n x n interior.  temp is n x n, compact. */         \
static void stencil_pass_##SUF(const AT *w, int n, const double taps[9], AT *temp)   \
{                                                                                    \
    int m = n + 2;                                                                   \
    AT t[9];                                                                         \
    for (int k = 0; k < 9; ++k) t[k] = (AT)taps[k];                                  \
    OX_ROWS                                                                          \
    for (int i = 1; i <= n; ++i)                                                     \
        for (int j = 1; j <= n; ++j) {                                               \
            AT acc = 0;                                                              \
            int first = 1;                                                           \
            for (int k = 0; k < 9; ++k) {                                            \
                int a = TAP_ORDER[k][0], b = TAP_ORDER[k][1];                        \
                AT tap = t[(a + 1) * 3 + (b + 1)];                                   \
                if (tap == 0) continue;                                              \
                AT term = tap * w[(size_t)(i + a) * m + (j + b)];                    \
                if (first) { acc = term; first = 0; }                                \
                else acc = acc + term;                                               \
            }                                                                        \
            temp[(size_t)(i - 1) * n + (j - 1)] = acc;                               \
        }                                                                            \
}                                                                                    \
                                                                                     \
/* Step 1 for the 5-point Laplacian (the filter t of the OL Laplace expression):    \
 * temp(i,j) = ((((N - 4C) + W) + E) + S), the generic pass above with the zero   \
 * taps dropped and the unit taps' exact multiplications left out. */             \
static void laplace_pass_##SUF(const AT *w, int n, AT *temp)                          \
{                                                                                    \
    int m = n + 2;                                                                   \
    OX_ROWS                                                                          \
    for (int i = 1; i <= n; ++i)                                                     \
        for (int j = 1; j <= n; ++j) {                                               \
            AT C = w[(size_t)i * m + j];                                             \
            AT N = w[(size_t)(i - 1) * m + j], S = w[(size_t)(i + 1) * m + j];       \
            AT W = w[(size_t)i * m + (j - 1)], E = w[(size_t)i * m + (j + 1)];       \
            temp[(size_t)(i - 1) * n + (j - 1)] = (((N - (AT)4 * C) + W) + E) + S;   \
        }                                                                            \
}                                                                                    \
                                                                                     \
/* Step 3 (OL max-norm): r = f - c*s over the interior; norms[0] = max|r| (NaN      \
 * propagating), norms[1] = sum r^2 in FP64, row-major order.  r_out optional;      \
 * rd_out (optional, n x n) receives each r as the FP64 number the norm squares.  */ \
static void norm_pass_##SUF(const AT *temp, int n, const ST *f, int ld_f, AT c,      \
                            ST *r_out, int ld_r, double *rd_out, double *norms)      \
{                                                                                    \
    double mx = 0.0, sq = 0.0;                                                       \
    for (int i = 0; i < n; ++i)                                                      \
        for (int j = 0; j < n; ++j) {                                                \
            AT r = LOAD(f[(size_t)i * ld_f + j]) - c * temp[(size_t)i * n + j];      \
            if (r_out) r_out[(size_t)i * ld_r + j] = STORE(r);                       \
            double rd = (double)r;                                                   \
            if (rd_out) rd_out[(size_t)i * n + j] = rd;                              \
            mx = nanmax_d(mx, fabs(rd));                                             \
            sq += rd * rd;                                                           \
        }                                                                            \
    if (norms) { norms[0] = mx; norms[1] = sq; }                                     \
}                                                                                    \
                                                                                     \
/* Output ghost ring of a freshly written phi_out, per side: odd reflection of the \
 * new interior (DIRICHLET0), the input's ghosts unchanged (GHOST_FIXED), or the   \
 * new interior n cells away (PERIODIC).  The four corner cells are left untouched \
 * except on a torus, where they are the opposite interior corners. */             \
static void write_out_ghosts_##SUF(const ST *in, ST *out, int n, int ld, const int bcs[4]) \
{                                                                                    \
    for (int k = 1; k <= n; ++k) {                                                   \
        size_t g[4] = {(size_t)0 * ld + k, (size_t)(n + 1) * ld + k,                 \
                       (size_t)k * ld + 0, (size_t)k * ld + n + 1};                  \
        size_t a[4] = {(size_t)1 * ld + k, (size_t)n * ld + k,                       \
                       (size_t)k * ld + 1, (size_t)k * ld + n};                      \
        size_t o[4] = {(size_t)n * ld + k, (size_t)1 * ld + k,                       \
                       (size_t)k * ld + n, (size_t)k * ld + 1};                      \
        for (int side = 0; side < 4; ++side)                                         \
            out[g[side]] = (bcs[side] == OX_BC_DIRICHLET0) ? STORE(-LOAD(out[a[side]])) \
                           : (bcs[side] == OX_BC_PERIODIC) ? out[o[side]]            \
                                                           : in[g[side]];            \
    }                                                                                \
    if (bcs[0] == OX_BC_PERIODIC && bcs[2] == OX_BC_PERIODIC) {                      \
        out[0] = out[(size_t)n * ld + n];                                            \
        out[n + 1] = out[(size_t)n * ld + 1];                                        \
        out[(size_t)(n + 1) * ld] = out[(size_t)1 * ld + n];                         \
        out[(size_t)(n + 1) * ld + n + 1] = out[(size_t)1 * ld + 1];                 \
    }                                                                                \
}                                                                                    \
                                                                                     \
/* Generic 3x3 stencil: out(i,j) = scale * S(phi)(i,j), out is n x ld_out. */        \
void ox_apply_stencil_##SUF(const ST *phi, int n, int ld, const double taps[9],      \
                            double scale, int bc, ST *out, int ld_out)               \
{                                                                                    \
    const int bcs[4] = {bc, bc, bc, bc};                                             \
    AT *w = ghosted_copy_##SUF(phi, n, ld, bcs);                                     \
    AT *temp = (AT *)malloc(sizeof(AT) * (size_t)n * n);                             \
    stencil_pass_##SUF(w, n, taps, temp);                                            \
    AT sc = (AT)scale;                                                               \
    for (int i = 0; i < n; ++i)                                                      \
        for (int j = 0; j < n; ++j)                                                  \
            out[(size_t)i * ld_out + j] = STORE(sc * temp[(size_t)i * n + j]);       \
    free(temp);                                                                      \
    free(w);                                                                         \
}                                                                                    \
                                                                                     \
/* Residual of phi: r = f - (1/h^2) S(phi); norms of r; r_out optional. */          \
static void residual_work_##SUF(const ST *phi, int n, int ld, const ST *f, int ld_f,  \
                                double h, const int bcs[4], ST *r_out, int ld_r,     \
                                double *rd_out, double *norms)                       \
{                                                                                    \
    AT c = (AT)(1.0 / (h * h));                                                      \
    AT *w = ghosted_copy_##SUF(phi, n, ld, bcs);                                     \
    AT *temp = (AT *)malloc(sizeof(AT) * (size_t)n * n);                             \
    laplace_pass_##SUF(w, n, temp);                                                  \
    norm_pass_##SUF(temp, n, f, ld_f, c, r_out, ld_r, rd_out, norms);                \
    free(temp);                                                                      \
    free(w);                                                                         \
}                                                                                    \
void ox_residual_sides_##SUF(const ST *phi, int n, int ld, const ST *f, int ld_f,    \
                             double h, const int bcs[4], ST *r_out, int ld_r,        \
                             double *norms)                                          \
{                                                                                    \
    residual_work_##SUF(phi, n, ld, f, ld_f, h, bcs, r_out, ld_r, NULL, norms);      \
}                                                                                    \
void ox_residual_##SUF(const ST *phi, int n, int ld, const ST *f, int ld_f,          \
                       double h, int bc, ST *r_out, int ld_r, double *norms)         \
{                                                                                    \
    const int bcs[4] = {bc, bc, bc, bc};                                             \
    ox_residual_sides_##SUF(phi, n, ld, f, ld_f, h, bcs, r_out, ld_r, norms);        \
}                                                                                    \
/* The residual of every interior cell as the FP64 number whose square the norm     \
 * adds (the arithmetic type's value, before any rounding to storage): rd_out is    \
 * n x n compact.  For an exact reference of the sum of squares. */                  \
void ox_residual_terms_##SUF(const ST *phi, int n, int ld, const ST *f, int ld_f,    \
                             double h, int bc, double *rd_out, double *norms)        \
{                                                                                    \
    const int bcs[4] = {bc, bc, bc, bc};                                             \
    residual_work_##SUF(phi, n, ld, f, ld_f, h, bcs, NULL, 0, rd_out, norms);        \
}                                                                                    \
                                                                                     \
/* One sweep in -> out (the three steps of the algorithm, then the output ghosts). \
 * norms (optional) receives the norm of the residual of the INPUT iterate. */      \
static void sweep_work_##SUF(const ST *in, ST *out, int n, int ld, const ST *f,      \
                             int ld_f, double h, double lambda, const int bcs[4],    \
                             double *norms, AT *w, AT *temp)                         \
{                                                                                    \
    AT c = (AT)(1.0 / (h * h));                                                      \
    AT wgt = (AT)(lambda / (h * h));                                                 \
    AT lam = (AT)lambda;                                                             \
    int m = n + 2;                                                                   \
    ghosted_fill_##SUF(in, n, ld, bcs, w);                                           \
    /* (1) Laplacian */                                                              \
    laplace_pass_##SUF(w, n, temp);                                                  \
    /* (2) Jacobi update (1, w, -lambda) on [phi; S phi; rho] */                     \
    OX_ROWS                                                                          \
    for (int i = 1; i <= n; ++i)                                                     \
        for (int j = 1; j <= n; ++j) {                                               \
            AT p = w[(size_t)i * m + j];                                             \
            AT s = temp[(size_t)(i - 1) * n + (j - 1)];                              \
            AT rho = LOAD(f[(size_t)(i - 1) * ld_f + (j - 1)]);                      \
            out[(size_t)i * ld + j] = STORE((p + wgt * s) - lam * rho);              \
        }                                                                            \
    /* (3) max-norm of the input iterate's residual */                               \
    if (norms) norm_pass_##SUF(temp, n, f, ld_f, c, NULL, 0, NULL, norms);           \
    write_out_ghosts_##SUF(in, out, n, ld, bcs);                                     \
}                                                                                    \
void ox_sweep_sides_##SUF(const ST *in, ST *out, int n, int ld, const ST *f,         \
                          int ld_f, double h, double lambda, const int bcs[4],       \
                          double *norms)                                             \
{                                                                                    \
    AT *w = (AT *)malloc(sizeof(AT) * (size_t)(n + 2) * (n + 2));                    \
    AT *temp = (AT *)malloc(sizeof(AT) * (size_t)n * n);                             \
    sweep_work_##SUF(in, out, n, ld, f, ld_f, h, lambda, bcs, norms, w, temp);       \
    free(temp);                                                                      \
    free(w);                                                                         \
}                                                                                    \
void ox_sweep_##SUF(const ST *in, ST *out, int n, int ld, const ST *f, int ld_f,     \
                    double h, double lambda, int bc, double *norms)                  \
{                                                                                    \
    const int bcs[4] = {bc, bc, bc, bc};                                             \
    ox_sweep_sides_##SUF(in, out, n, ld, f, ld_f, h, lambda, bcs, norms);            \
}                                                                                    \
                                                                                     \
/* nsweeps sweeps in -> out (in is not modified; out gets the final iterate).       \
 * resmode LAGGED: norms of the last sweep's input; FINAL: norms of out.            \
 * nsweeps == 0 copies in to out.  The four corner cells of out are not written   \
 * (the 5-point stencil does not read them), except on a torus (all sides          \
 * PERIODIC), where they are the opposite interior corners.  bcs: per-side modes  \
 * (north, south, west, east); a GHOST_FIXED side models a box interface whose    \
 * ghost layer was filled from a neighbouring box before the sweeps. */           \
void ox_relax_sides_##SUF(const ST *in, ST *out, int n, int ld, const ST *f,         \
                          int ld_f, double h, double lambda, int nsweeps,            \
                          const int bcs[4], int resmode, double *norms)              \
{                                                                                    \
    int m = n + 2;                                                                   \
    size_t total = (size_t)(m - 1) * ld + m;                                         \
    ST *a = (ST *)malloc(sizeof(ST) * total);                                        \
    ST *b = (ST *)malloc(sizeof(ST) * total);                                        \
    memcpy(a, in, sizeof(ST) * total);                                               \
    memcpy(b, in, sizeof(ST) * total);                                               \
    /* work arrays of the sweeps, allocated once */                                  \
    AT *w = (AT *)malloc(sizeof(AT) * (size_t)m * m);                                \
    AT *temp = (AT *)malloc(sizeof(AT) * (size_t)n * n);                             \
    for (int it = 0; it < nsweeps; ++it) {                                           \
        double *nrm = (resmode == OX_RES_LAGGED && it == nsweeps - 1) ? norms : NULL;\
        sweep_work_##SUF(a, b, n, ld, f, ld_f, h, lambda, bcs, nrm, w, temp);        \
        ST *t = a; a = b; b = t;                                                     \
    }                                                                                \
    free(temp);                                                                      \
    free(w);                                                                         \
    const int torus = bcs[0] == OX_BC_PERIODIC && bcs[2] == OX_BC_PERIODIC;         \
    OX_ROWS                                                                          \
    for (int i = 0; i < m; ++i)                                                      \
        for (int j = 0; j < m; ++j) {                                                \
            int corner = (i == 0 || i == m - 1) && (j == 0 || j == m - 1);           \
            if (!corner || (torus && nsweeps > 0)) out[(size_t)i * ld + j] = a[(size_t)i * ld + j]; \
        }                                                                            \
    if (resmode == OX_RES_FINAL)                                                     \
        ox_residual_sides_##SUF(a, n, ld, f, ld_f, h, bcs, NULL, 0, norms);          \
    free(a);                                                                         \
    free(b);                                                                         \
}                                                                                    \
void ox_relax_##SUF(const ST *in, ST *out, int n, int ld, const ST *f, int ld_f,     \
                    double h, double lambda, int nsweeps, int bc, int resmode,       \
                    double *norms)                                                   \
{                                                                                    \
    const int bcs[4] = {bc, bc, bc, bc};                                             \
    ox_relax_sides_##SUF(in, out, n, ld, f, ld_f, h, lambda, nsweeps, bcs, resmode,  \
                         norms);                                                     \
}

#define ID(x) (x)
OX_DEFINE(f64, double, double, ID, ID)
OX_DEFINE(f32, float, float, ID, ID)
OX_DEFINE(bf16, uint16_t, float, ox_bf16_to_f32, ox_f32_to_bf16)

/* ================================================================== */
/* Mixed-precision iterative refinement (an extension beyond the paper: */
/* the relaxation of the paper run on the error equation).              */
/*                                                                      */
/* Outer step in FP64:   r = f - L phi  (the FP64 residual above),      */
/*                       stop when max|r| <= rtol * max|f|;             */
/* inner solve in low precision:  L delta = r  by k_in plain Jacobi     */
/*                       sweeps from delta = 0 (storage per variant);   */
/* update in FP64:       phi = phi + delta.                             */
/* lowp: 1 = FP32 storage and arithmetic, 2 = BF16 storage, FP32 math.  */
/* Returns the number of outer steps taken; norms of the last residual  */
/* in norms[0..1]; phi is updated in place.                             */
/* ================================================================== */
int ox_refine(double *phi, int n, int ld, const double *f, int ld_f, double h,
              double lambda, int bc, int lowp, int k_in, int max_outer,
              double rtol, double *norms)
{
    int m = n + 2;
    size_t total = (size_t)(m - 1) * ld + m;
    double fmax = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) fmax = nanmax_d(fmax, fabs(f[(size_t)i * ld_f + j]));
    double *r = (double *)malloc(sizeof(double) * (size_t)n * n);
    /* low-precision buffers: delta (ghosted, same ld) and its right-hand side */
    void *d_in = calloc(total, lowp == 1 ? 4 : 2);
    void *d_out = calloc(total, lowp == 1 ? 4 : 2);
    void *rl = calloc((size_t)n * n, lowp == 1 ? 4 : 2);
    int outer = 0;
    for (;;) {
        ox_residual_f64(phi, n, ld, f, ld_f, h, bc, r, n, norms);
        int converged = norms[0] <= rtol * fmax;
        if (converged || isnan(norms[0]) || outer >= max_outer) break;
        /* r rounded into the inner right-hand side: FP64 -> FP32 (-> BF16) */
        OX_ROWS
        for (size_t q = 0; q < (size_t)n * n; ++q) {
            if (lowp == 1) ((float *)rl)[q] = (float)r[q];
            else ((uint16_t *)rl)[q] = ox_f32_to_bf16((float)r[q]);
        }
        /* delta starts at zero, ghosts included (the error of a fixed ghost is 0) */
        memset(d_in, 0, total * (lowp == 1 ? 4 : 2));
        if (lowp == 1)
            ox_relax_f32((const float *)d_in, (float *)d_out, n, ld, (const float *)rl, n,
                         h, lambda, k_in, bc, OX_RES_NONE, NULL);
        else
            ox_relax_bf16((const uint16_t *)d_in, (uint16_t *)d_out, n, ld,
                          (const uint16_t *)rl, n, h, lambda, k_in, bc, OX_RES_NONE, NULL);
        OX_ROWS
        for (int i = 1; i <= n; ++i)
            for (int j = 1; j <= n; ++j) {
                size_t q = (size_t)i * ld + j;
                double dv = (lowp == 1) ? (double)((float *)d_out)[q]
                                        : (double)ox_bf16_to_f32(((uint16_t *)d_out)[q]);
                phi[q] = phi[q] + dv;
            }
        ++outer;
    }
    free(r);
    free(d_in);
    free(d_out);
    free(rl);
    return outer;
}

/* Array form of the bfloat16 rounding above (for preparing test inputs). */
void ox_f32_to_bf16_array(const float *x, uint16_t *y, size_t count)
{
    for (size_t q = 0; q < count; ++q) y[q] = ox_f32_to_bf16(x[q]);
}
