/*
 * protox.h -- C ABI of the MI355X (gfx950) fused Poisson relaxation library.
 *
 * The operations follow Section IV of the ProtoX paper ("2D Poisson
 * equation", "Algorithm", the OL expressions and the generated fused code):
 *
 *   stencil    S(phi)(i,j) = sum_{a,b in -1..1} t[a][b] phi(i+a, j+b)   (Eq. 1)
 *              with the 5-point filter t = [0,1,0; 1,-4,1; 0,1,0];
 *   Laplacian  L = S / h^2, the discretisation of Eq. 2;
 *   Jacobi     phi' = (phi + w s) - lambda f,  s = S(phi), w = lambda / h^2
 *              (Eq. 3 in the OL form (1, w, -lambda) on [phi; S phi; rho]);
 *   residual   r = f - (1/h^2) s, reported as max|r| (the max-norm of the
 *              OL norm expression; NaN-propagating) and sum r^2.
 *
 * The right-hand side is called f here (rho in the paper).
 *
 * Data layout (all grids row-major, column index fastest):
 *   phi  (n+2) rows x ld elements, ld >= n+2; interior cells at rows and
 *        columns 1..n, one ghost layer around them.  The buffer must hold
 *        (n+2)*ld elements.
 *   f    n rows x ld_f elements, ld_f >= n; f[(i-1)*ld_f + (j-1)] belongs to
 *        phi cell (i, j).  The buffer must hold n*ld_f elements.
 *   out/r/temp of stencil and residual calls: n rows x ld_x, compact like f.
 * Grid spacing h = 1/n for the cell-centred unit square (the caller passes h).
 *
 * Boundary handling (px_bc):
 *   PX_BC_DIRICHLET0   homogeneous Dirichlet at the cell faces: every sweep
 *                      reads ghost = -(adjacent interior) (odd reflection),
 *                      whatever the ghost ring holds; outputs of relax calls
 *                      get their edge ghosts written the same way.
 *   PX_BC_GHOST_FIXED  the ghost ring is read as given and never changes
 *                      (the paper's generated code reads ghosts and never
 *                      writes them); relax copies it to the output.
 *   The four corner cells of a phi output are never written (the 5-point
 *   stencil does not read them).  For general 3x3 taps under DIRICHLET0 the
 *   corner ghost is +(diagonal interior) (reflection in both directions).
 *
 * Element types (px_dtype): FP64, FP32, BF16 (bfloat16 storage, FP32
 * arithmetic, round-to-nearest-even on every store).  Arithmetic follows the
 * association above with every operation rounded on its own, so results are
 * reproducible bit for bit (the fused relaxation forms N - 4C as one fused
 * multiply-add, which rounds the same exact value while 4|C| is finite); the
 * FP32/BF16 constants w, 1/h^2 and lambda are computed in FP64 and rounded
 * once.
 *
 * Ownership and ordering: every pointer argument named as device memory is
 * owned by the caller and never freed by the library.  Calls enqueue work on
 * `stream` (a hipStream_t; NULL = the default stream) and return without
 * waiting, except px_solve, which waits on the stream to read norms.
 * A px_ctx owns scratch device memory (ping-pong grid, reduction partials)
 * and must not be used by two calls that may run concurrently.
 *
 * Errors: every function returns a px_status.  Arguments are validated on
 * the host before any HIP call; on failure nothing is enqueued and
 * px_last_error() (thread-local) describes the problem.  HIP failures map to
 * PX_EHIP.  No exception or abort crosses this interface.
 */
#ifndef PROTOX_H
#define PROTOX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum px_status {
    PX_OK = 0,
    PX_EINVAL = -1,        /* bad size, pointer, alignment, enum or value    */
    PX_EUNSUPPORTED = -2,  /* valid request the library does not implement  */
    PX_EALIAS = -3,        /* an output overlaps an input it must not alias  */
    PX_EHIP = -4,          /* the HIP runtime reported an error              */
    PX_ENOTCONV = -5,      /* px_solve: max_sweeps reached before tolerance  */
    PX_EDIVERGED = -6,     /* px_solve: residual grew beyond recovery        */
    PX_ENONFINITE = -7,    /* px_solve: NaN or Inf in the residual           */
    PX_ENOMEM = -8         /* scratch allocation failed                      */
} px_status;

typedef enum px_dtype { PX_F64 = 0, PX_F32 = 1, PX_BF16 = 2 } px_dtype;
typedef enum px_bc {
    PX_BC_DIRICHLET0 = 0,  /* homogeneous Dirichlet at the cell faces: odd reflection,
                              ghost := -(adjacent interior) at every sweep             */
    PX_BC_GHOST_FIXED = 1, /* the ghost ring is read as given and never changed       */
    PX_BC_PERIODIC = 2     /* torus (Proto's own boundary, Section II): a ghost is the
                              interior cell n cells away; outputs write the ghost ring
                              and its corners.  Stencil, residual, relaxation, autotune
                              and plain solves only (PX_EUNSUPPORTED elsewhere); a
                              solvable system needs f with zero sum                     */
} px_bc;
typedef enum px_resmode {
    PX_RES_NONE = 0,   /* no norms                                              */
    PX_RES_LAGGED = 1, /* norms of the residual of the LAST sweep's input, the  */
                       /* quantity the paper's fused loop computes              */
    PX_RES_FINAL = 2   /* norms of the residual of phi_out (the Proto order)    */
} px_resmode;

typedef struct px_ctx px_ctx;

/* Context on HIP device `device`; *out receives it.  Allocates nothing yet. */
int px_ctx_create(int device, px_ctx **out);
/* Frees the context's scratch (waits for the device first). NULL is a no-op. */
int px_ctx_destroy(px_ctx *ctx);
/* Pre-allocates the scratch a relax/solve call on an (n, ld, dtype) grid
 * needs, so that later calls allocate nothing. */
int px_ctx_reserve(px_ctx *ctx, int n, int ld, int dtype);
/* Rows per tile of the fused relaxation kernel (0 = built-in heuristic).
 * A tuning knob; any value in [1, 4096] gives identical results. */
int px_ctx_set_tile_rows(px_ctx *ctx, int rows);

/*
 * Autotuner: times the fused relaxation on the caller's buffers for every
 * sweeps-per-launch k in 1..8 and a list of tile heights (for k = 2, 5, 8
 * those from 16 rows up rounded up to fill the unrolled loop's blocks of
 * k + 1 steps; fastest of five single launches each), re-times the four best
 * as runs of 24 launches that each read the previous one's output (as a sweep
 * loop runs them), gives the two best of those a tile height for their
 * launches that also take the residual norms (fastest of three launches per
 * height), times both as whole calls (24 launches, the last with norms;
 * median of five) and remembers the faster (within 1.5% at equal k: the
 * taller band) in ctx for
 * this (dtype, n, ld).  Later calls with tblock == 0 on such a grid use them
 * (explicit tblock or px_ctx_set_tile_rows override them).  phi_in is only
 * read; phi_out is overwritten with scratch iterates; f as in px_relax_fused.
 * Allocates the context's ping-pong grid.  Waits on `stream`.  best_k,
 * best_rows and gcells (cell-updates per second / 1e9 of the winner) may be
 * NULL.
 */
int px_autotune(const void *phi_in, void *phi_out, int n, int ld, int dtype, const void *f,
                int ld_f, int bc, px_ctx *ctx, void *stream, int *best_k, int *best_rows,
                double *gcells);

/* Message of the last failing call on this thread ("" if none). */
const char *px_last_error(void);
const char *px_version(void);

/*
 * Stencil (Eq. 1): out(i,j) = scale * S(phi)(i,j) for the n x n interior,
 * taps[3*(a+1) + (b+1)] = t[a][b] (host array of 9 doubles, row a = -1 is
 * the row above).  Taps are visited in the order (-1,0), (0,0), (0,-1),
 * (0,1), (1,0), then the corners; zero taps are skipped, so for the 5-point
 * Laplacian the sum is ((((N - 4C) + W) + E) + S), the order of the paper's
 * generated code.  scale == 1 skips the multiplication.
 * phi: device, (n+2) x ld; out: device, n x ld_out.  phi and out must not
 * overlap (PX_EALIAS).
 */
int px_apply_stencil(const void *phi, int n, int ld, int dtype, void *out, int ld_out,
                     const double *taps, double scale, int bc, void *stream);

/*
 * Residual (the OL max-norm expression): r = f - (1/h^2) S(phi) over the
 * interior, S the 5-point stencil.  r (device, n x ld_r, same dtype; may be
 * NULL) receives the residual; norms (device, 2 doubles) receives
 * { max|r|, sum r^2 }, both accumulated in FP64 (max NaN-propagating).
 * Needs ctx for reduction scratch.
 */
int px_residual(const void *phi, int n, int ld, int dtype, const void *f, int ld_f, double h,
                int bc, void *r, int ld_r, double *norms, px_ctx *ctx, void *stream);

/*
 * The pointwise Jacobi step on its own (the unfused form, Proto's
 * forallInPlace): phi(i,j) = (phi(i,j) + w s(i,j)) - lambda f(i,j) in place
 * over the interior, with s (device, n x ld_s) the unscaled stencil of phi
 * from px_apply_stencil and w = lambda / h^2.  Ghosts are not touched.
 */
int px_jacobi_update(void *phi, int n, int ld, int dtype, const void *s, int ld_s,
                     const void *f, int ld_f, double h, double lambda, void *stream);

/*
 * Fused relaxation (Section IV: the Jacobi step of Eq. 3 with the stencil of
 * Eq. 1, fused with the max-norm as in the generated CPU loop of Fig. 5 and
 * the GPU kernel of Fig. 7, which compute the update and the norm in one pass
 * over the grid): nsweeps damped-Jacobi sweeps phi_in -> phi_out, each
 * sweep computing the stencil, the update and (on the sweep resmode asks
 * for) the residual norms in one pass over memory.  Several sweeps run per
 * kernel launch (temporal blocking): tblock in 1..8 sweeps per launch, 0 =
 * library default.  Results do not depend on tblock or on the tile shape.
 * phi_in is read-only; phi_out receives the final iterate, its edge ghosts
 * per bc; both (n+2) x ld of dtype, non-overlapping (PX_EALIAS); f must not
 * overlap phi_out.  nsweeps == 0 copies phi_in to phi_out (corners
 * excepted).  norms: device, 2 doubles, required unless resmode is
 * PX_RES_NONE.  Needs ctx (ping-pong buffer when more than one launch is
 * needed, reduction partials).
 */
int px_relax_fused(const void *phi_in, void *phi_out, int n, int ld, int dtype, const void *f,
                   int ld_f, double h, double lambda, int nsweeps, int tblock, int bc,
                   int resmode, double *norms, px_ctx *ctx, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one launch of
 * px_relax_fused -- 1 <= nsweeps <= 8 sweeps, temporally blocked in a single
 * kernel launch, default tile height -- with no context.  Same arguments,
 * results and errors as px_relax_fused otherwise (bit-identical outputs and
 * norms).  Longer runs alternate phi_in/phi_out buffers of the caller's own.
 * The reduction partials live in a fixed device array of the library
 * (PX_NOALLOC_MAX_PARTIALS slots of 16 bytes = 2 MiB on every GPU the call
 * runs on, held until the process ends); grids needing more partials than it
 * holds are rejected with PX_EINVAL (every grid up to n = 16384 fits).  Runs on
 * the current HIP device.  Calls that overlap on one GPU race on that array:
 * serialise them (one stream, or events).  Allocates nothing: the first call
 * on a device only looks the array's address up.
 */
#define PX_NOALLOC_MAX_PARTIALS (1 << 17)
int px_relax_fused_noalloc(const void *phi_in, void *phi_out, int n, int ld, int dtype, const void *f,
                           int ld_f, double h, double lambda, int nsweeps, int bc, int resmode,
                           double *norms, void *stream);

/* ---------------------------------------------------------------------- */
/* Iterative solve (the paper's Algorithm iterated to a tolerance).         */
/* ---------------------------------------------------------------------- */
typedef enum px_mode {
    PX_SOLVE_PLAIN = 0,      /* fused relaxation in phi's own precision           */
    PX_SOLVE_MIXED_F32 = 1,  /* FP64 refinement around FP32 inner sweeps          */
    PX_SOLVE_MIXED_BF16 = 2  /* FP64 refinement around BF16-storage inner sweeps  */
} px_mode;

typedef struct px_solve_opts {
    int mode;              /* px_mode                                            */
    int norm;              /* 0: stop on max-norm, 1: on the L2 norm             */
    double rtol;           /* stop when ||r|| <= rtol * ||f|| (same norm)        */
    int64_t max_sweeps;    /* sweep budget (inner sweeps for MIXED modes)        */
    int check_every;       /* sweeps between residual checks (PLAIN); MIXED modes
                              read the norms back every check_every / inner_sweeps
                              outer steps (at least every step)                  */
    int inner_sweeps;      /* sweeps per inner solve (MIXED); 0 = default:
                              1024 (FP32) or 128 (BF16)                          */
    int tblock;            /* sweeps per launch, 0 = default                     */
    int bc;                /* px_bc                                              */
} px_solve_opts;

typedef struct px_solve_stats {
    int64_t sweeps;        /* sweeps performed                                   */
    int64_t outer_steps;   /* refinement steps (MIXED) or checks (PLAIN)         */
    double res_max;        /* final max|r|                                       */
    double res_l2;         /* final sqrt(sum r^2)                                */
    double rel_res_max;    /* res_max / max|f|                                   */
    double rel_res_l2;     /* res_l2 / ||f||_2                                   */
    double seconds;        /* host wall time inside px_solve                     */
} px_solve_stats;

/*
 * Solve L phi = f from the given phi (in place, FP64 storage for the MIXED
 * modes, any dtype for PLAIN), stopping at the tolerance, on NaN/Inf
 * (PX_ENONFINITE), on growth of the residual by 1e8 over its start
 * (PX_EDIVERGED) or at max_sweeps (PX_ENOTCONV).  f is in phi's dtype
 * (FP64 for MIXED).  Waits on `stream` at every check.  stats may be NULL.
 */
int px_solve(void *phi, int n, int ld, int dtype, const void *f, int ld_f, double h,
             double lambda, const px_solve_opts *opts, px_solve_stats *stats, px_ctx *ctx,
             void *stream);

/* ---------------------------------------------------------------------- */
/* Batches of independent problems (not in the paper: many Poisson problems */
/* of uneven sizes solved together).                                        */
/* ---------------------------------------------------------------------- */
typedef struct px_problem {
    void *phi;        /* device, (n+2) x ld: initial iterate in, result out (in place) */
    const void *f;    /* device, n x ld_f                                              */
    int n, ld, ld_f;
    double h, lambda; /* as for px_relax_fused                                         */
} px_problem;

/*
 * nsweeps fused sweeps on every problem of the batch (all of element type
 * dtype and boundary mode bc), in place.  One persistent kernel launch per
 * tblock sweeps walks the tiles of all problems; intermediate iterates live in
 * ctx-owned memory.  norms (device, 2*nprob doubles) receives each problem's
 * {max|r|, sum r^2} of its final iterate when resmode is PX_RES_FINAL (other
 * modes: no norms; norms may be NULL).  probs is a host array.  Every phi and f
 * must start 16-byte aligned with ld and ld_f multiples of 16 bytes
 * (PX_EINVAL otherwise); the problems' phi must not overlap (PX_EALIAS).
 */
int px_relax_batched(const px_problem *probs, int nprob, int dtype, int nsweeps, int tblock, int bc,
                     int resmode, double *norms, px_ctx *ctx, void *stream);

/*
 * One domain split into boxes (Section IV: the grid is a union of boxes, each with its
 * own ghost layer, and a sweep first fills every box's ghost cells from its neighbours'
 * interiors, then relaxes each box on its own): nbx x nby boxes of n x n cells, boxes[i]
 * for box row i / nbx and box column i % nbx (box (r, c) holds domain rows r*n .. r*n+n-1
 * and columns c*n .. c*n+n-1), each with its own phi ((n+2) x ld, in place) and f; every
 * box has the same n, h and lambda.  Every `exchange` sweeps (1..8; nsweeps must be a
 * multiple) the ghost ring of every box is refreshed: a side facing another box takes that
 * box's adjacent interior row or column; a side on the domain's edge takes -(adjacent
 * interior) under PX_BC_DIRICHLET0, wraps onto the opposite edge's box under
 * PX_BC_PERIODIC, and keeps its values under PX_BC_GHOST_FIXED.  Then every box relaxes
 * `exchange` sweeps with its ghost ring held fixed (interface values lag by up to
 * exchange - 1 sweeps).  With exchange = 1 the boxes' interiors equal px_relax_fused on the
 * whole domain bit for bit.  Corners are not written.  Alignment and aliasing rules as for
 * px_relax_batched; at most 65535 boxes.  Needs ctx (scratch of the batched relaxation).
 */
int px_relax_boxes(const px_problem *boxes, int nbx, int nby, int dtype, int nsweeps, int exchange, int bc,
                   px_ctx *ctx, void *stream);

/*
 * Autotuner for batches: the tile rows of each problem size (the problems of that size
 * relaxed alone with the persistent kernel, 8 sweeps per launch, every candidate height),
 * then the sweeps per launch k in 1..8 for the whole batch.  Remembered in ctx for
 * dtype: px_relax_batched (dtype) and px_solve_batched (inner sweeps of that dtype:
 * PX_F32 for PX_SOLVE_MIXED_F32, PX_BF16 for PX_SOLVE_MIXED_BF16) use them when tblock
 * is 0 (px_ctx_set_tile_rows still overrides the rows).  Any dtype's results are
 * identical with or without tuning.  The problems are relaxed IN PLACE while timing
 * (their phi is overwritten): pass scratch problems of the same sizes, or
 * re-initialise them afterwards.  Waits on `stream`.  best_k may be NULL.
 */
int px_autotune_batched(const px_problem *probs, int nprob, int dtype, int bc, px_ctx *ctx, void *stream,
                        int *best_k);

/*
 * Solve every problem of the batch to its tolerance with FP64 iterative
 * refinement around low-precision inner sweeps (opts->mode PX_SOLVE_MIXED_F32
 * or PX_SOLVE_MIXED_BF16; phi and f are FP64; the arithmetic is that of
 * px_solve with the same mode, inner_sweeps and tblock, so every problem's
 * result equals its single-problem solve).  One outer step of the whole batch
 * is captured once as a hipGraph and replayed; problems that converge are
 * switched off on the device.  stats: host array of nprob entries (may be
 * NULL); .seconds is the wall time of the whole batch.  Returns PX_OK when
 * every problem converged, else the status of the first that did not.
 * Waits on `stream`.
 */
int px_solve_batched(const px_problem *probs, int nprob, const px_solve_opts *opts, px_solve_stats *stats,
                     px_ctx *ctx, void *stream);

/* ---------------------------------------------------------------------- */
/* Learned correction network (not in the paper: a small convolutional     */
/* network that maps a residual to a correction inside a refinement loop). */
/* ---------------------------------------------------------------------- */
/*
 * Architecture: x -> conv3x3(1->32) -> ReLU -> conv3x3(32->32) -> ReLU ->
 * conv3x3(32->32) -> ReLU -> conv3x3(32->1) -> y; no bias; zero padding (every
 * activation is 0 outside the image).  Weights: PX_NET_NPARAM FP32 numbers, the
 * four layers in order, each in (out, in, 3, 3) C order.  Arithmetic: the input,
 * the weights and every hidden activation are rounded to bfloat16 (nearest, ties
 * to even); sums accumulate in FP32 (the 32->32 layers on the matrix cores).
 * Images: `batch` images of H x W pixels, row-major, FP32 unless stated.
 */
#define PX_NET_NPARAM 19008

typedef struct px_net px_net;

typedef enum px_loss {
    PX_LOSS_MSE = 0,    /* mean over pixels of (y - t)^2                                  */
    PX_LOSS_ENERGY = 1  /* mean over pixels of (y - t) K (y - t), K = 4 I - (4 neighbours),
                           odd reflection at the image edges (the negated 5-point stencil
                           under PX_BC_DIRICHLET0): the energy norm of the error           */
} px_loss;

/* Network on `device` with the given initial weights (host array of
 * PX_NET_NPARAM); optimiser state (Adam moments, step count) starts at zero. */
int px_net_create(int device, const float *weights, px_net **out);
int px_net_destroy(px_net *net);
/* Replace the weights (host array) and reset the optimiser state.  Waits. */
int px_net_set_weights(px_net *net, const float *weights);
/* Copy the FP32 master weights to a host array of PX_NET_NPARAM.  Waits. */
int px_net_get_weights(px_net *net, float *weights);

/*
 * y = N(x * x_scale) for `batch` images.  x: device, x_dtype PX_F64 or PX_F32,
 * image b row i at x + (b*H + i)*ldx (ldx >= W); y: device FP32, rows of ldy >= W.
 * The scaled input is rounded to bfloat16 as the first layer's input.
 */
int px_net_forward(px_net *net, const void *x, int x_dtype, int ldx, int batch, int H, int W,
                   double x_scale, float *y, int ldy, void *stream);

/*
 * One training evaluation on inputs x and targets t (device, FP32, compact
 * batch x H x W): forward pass, loss (px_loss), backward pass.  The gradient with
 * respect to the FP32 weights is kept in the network for px_net_adam and, when
 * grad is not NULL, copied to grad (device, PX_NET_NPARAM floats).  When loss_out
 * is not NULL (device, one double) it receives the loss.  The loss and every
 * gradient are reduced in a fixed order: results are reproducible bit for bit.
 */
int px_net_loss_grad(px_net *net, const float *x, const float *t, int batch, int H, int W, int loss,
                     double *loss_out, float *grad, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
 * gradient of the last px_net_loss_grad call, then re-rounds the bfloat16 copies. */
int px_net_adam(px_net *net, float lr, void *stream);

/*
 * The same y as px_net_forward, bit for bit, for inference: the first two layers run as
 * one kernel that computes layer 1 on the fly into the second layer's input patches, so
 * the 64-byte-per-pixel layer-1 activations never go through memory.  The hidden
 * activations are not kept (px_net_activation then fails until the next
 * px_net_forward).  The learned refinement loop evaluates the network this way.
 */
int px_net_infer(px_net *net, const void *x, int x_dtype, int ldx, int batch, int H, int W,
                 double x_scale, float *y, int ldy, void *stream);

/* Copy the hidden activation of layer 1, 2 or 3 of the last forward pass
 * (bfloat16 bit patterns, channels last: batch*H*W*32 values) to out (device). */
int px_net_activation(px_net *net, int layer, uint16_t *out, void *stream);

/*
 * A training pair from an iterate phi ((n+2) x ld FP64, device) of the
 * homogeneous problem L phi = 0 under PX_BC_DIRICHLET0, whose exact solution is
 * 0: error e = -phi and residual r = -L phi.  Writes x = r / rms(r) and the target
 * t = e / rms(e) (PX_LOSS_MSE) or t = e / sqrt(mean(e K e)) (PX_LOSS_ENERGY), as
 * compact n x n FP32 (device).  Scale factors 1/h^2 cancel, so h is not needed.
 * A field that is identically zero is written as zeros.  Uses ctx scratch.
 */
int px_net_make_pair(const double *phi, int n, int ld, int loss, float *x, float *t, px_ctx *ctx,
                     void *stream);

typedef struct px_learned_opts {
    int norm;             /* 0: stop on max-norm, 1: on the L2 norm                    */
    double rtol;          /* stop when ||r|| <= rtol * ||f|| (same norm)               */
    int64_t max_sweeps;   /* budget of relaxation sweeps                               */
    int smooth_sweeps;    /* plain sweeps after each correction (>= 1)                 */
    int tblock;           /* sweeps per launch, 0 = default                            */
    int use_net;          /* correction directions: 0: r alone (the same loop without
                             the network); 1: N(r / rms(r)) alone; 2: both, combined
                             as px_correction_step mode 2                              */
    int judge;            /* what a finite step that raised the residual triggers:
                             0: nothing (every finite step is kept); 1: the step is
                             kept, plain steps follow for a back-off period; 2: the
                             step is undone, plain steps follow for a back-off period */
} px_learned_opts;

typedef struct px_learned_stats {
    px_solve_stats base;  /* sweeps, outer_steps (= steps of the loop), norms, time    */
    int64_t corrections;  /* correction steps kept                                     */
    int64_t rejected;     /* correction steps undone by the judge                      */
    int fell_back;        /* 1 when a non-finite step switched corrections off         */
    int64_t discarded_sweeps; /* smoothing sweeps of undone steps: run, then discarded
                                 with the step; included in base.sweeps and counted
                                 against max_sweeps                                  */
} px_learned_stats;

/*
 * One correction step of the learned refinement (not in the paper): phi += a r + b d
 * over the interior of phi ((n+2) x ld FP64, device, in place), with (a, b) chosen to
 * minimise the energy norm <e, -L e> of the error e = L^-1 r after the step over the
 * directions `mode` allows: 0: r alone (b = 0; d may be NULL); 1: d alone (a = 0);
 * 2: both.  That is the Galerkin condition c M (a, b) = (<r,r>, <d,r>) with
 * M = [<r,Sr> <r,Sd>; <r,Sd> <d,Sd>], c = 1/h^2, S the 5-point stencil with odd
 * reflection (PX_BC_DIRICHLET0); a zero denominator gives a zero coefficient and a
 * numerically singular M (|det| <= 1e-10 |<r,Sr><d,Sd>|) falls back to mode 0.
 * r: device FP64 n x ld_r, the residual f - L phi; d: device n x ld_d, d_dtype PX_F64
 * or PX_F32.  coef (device, 2 doubles, may be NULL) receives (a, b).  Dot products are
 * FP64 in a fixed order.  phi must not overlap r or d (PX_EALIAS).
 */
int px_correction_step(void *phi, int n, int ld, const double *r, int ld_r, const void *d, int d_dtype, int ld_d,
                       double h, int mode, double *coef, px_ctx *ctx, void *stream);

/*
 * Solve L phi = f (FP64 phi and f, PX_BC_DIRICHLET0) by a refinement loop.  Each
 * step: r = f - L phi in FP64; the correction step of px_correction_step with
 * d = N(r / rms(r)) and mode = use_net (FP64 update); then smooth_sweeps fused
 * relaxation sweeps.  Plain
 * relaxation judges each step by its FP64 residual.  If the L2 norm after the step
 * (and its sweeps) is not finite (a broken network) the step is undone and the solve
 * continues with plain relaxation alone, which then equals the loop of px_solve
 * PX_SOLVE_PLAIN with check_every = smooth_sweeps.  If it is finite but not below the
 * norm before, opts->judge decides: keep the step (0), keep it and relax plainly for
 * the next 1, 2, 4, ... steps (1), or undo it and do the same (2); the back-off period
 * doubles while steps keep failing (at most 64) and resets when one succeeds.  Every
 * step with a finite result lowers the energy norm of the error (the step minimises it
 * over its directions, which include the zero step, and damped Jacobi sweeps with
 * omega <= 1 never raise it), so keeping such steps is safe.  Stopping rules
 * and return codes as px_solve.  Waits on `stream` every step.  net may be NULL when
 * use_net is 0.  stats may be NULL.
 */
int px_solve_learned(void *phi, int n, int ld, const double *f, int ld_f, double h, double lambda,
                     px_net *net, const px_learned_opts *opts, px_learned_stats *stats, px_ctx *ctx,
                     void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PROTOX_H */
