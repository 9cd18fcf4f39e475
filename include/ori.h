/*
 * ori.h -- C ABI of the MI355X (gfx950) solver for the reduced linear system
 * of Ramm & Tran, "A Fast Algorithm for Solving Scalar Wave Scattering
 * Problem by Billions of Particles" (arXiv:1602.04691).
 *
 * The system (Section 2, eq. 2.19, with c_S = 4 pi for spheres):
 *
 *     u_q + sum_{p != q} G(x_q, x_p) D_p u_p = u0_q,     q = 0 .. P-1,
 *     G(x, y) = exp(i k |x - y|) / (4 pi |x - y|)           (eq. 2.6a)
 *     D_p     = 4 pi h_p N_p |Delta_p|,  |Delta_p| = (side/n)^3,
 *
 * on the n^3 cubes Delta_p of the cube [origin, origin + side]^3, with the
 * point x_p = origin + side * (i + cell_offset) / n of each cube
 * (cell_offset = 0.5: centres, eqs. 2.18-2.19; 0: the lattice of eq. 3.3.5).
 * It is solved by COCG (van der Vorst & Melissen; cited in Sections 1 and 3)
 * whose products with the Green's matrix are 3-D convolutions evaluated with
 * FFTs after zero padding (Section 3, eqs. 3.3.4-3.3.8): here on a (2n)^3
 * grid with a precomputed kernel spectrum.
 *
 * Conventions (all entry points):
 *  - Flat index p = (i1 * n + i2) * n + i3, i3 fastest.  P = n^3.
 *  - Complex arrays are interleaved {re, im} doubles (C99 double complex,
 *    torch.complex128), 16-byte aligned; real arrays (N, points,
 *    directions) are doubles, 8-byte aligned.
 *  - Every array argument is DEVICE memory of the current HIP device
 *    (hipMalloc / torch CUDA tensors).  Host pointers are rejected with
 *    ORI_ERR_INVALID_ARG before any kernel runs.  Structs (ori_grid,
 *    ori_solve_opts, ori_solve_info) are host memory.
 *  - Caller buffers are never retained: ori_load copies what it needs.
 *  - All device work is ordered on the stream given to ori_create /
 *    ori_setup (NULL: the null stream); every call returns after that work
 *    has completed.
 *  - Errors are status codes; nothing aborts or throws across the ABI.
 *    ori_last_error(ctx) gives a text.  After ORI_ERR_DEVICE the context is
 *    poisoned: only ori_destroy is valid.
 *  - A context is not thread safe; distinct contexts are independent.
 *  - Supported n: every 1 <= n <= 512.  Each axis is padded to the
 *    shortest planned FFT length L >= 2n - 1 from
 *    {2,4,6,8,10,12,16,20,24,32,40,48,64,80,96,128,192,256,384,512,1024}
 *    (the cyclic convolution of length L then holds every offset in
 *    (-n, n): Section 3's zero padding); L = 2n whenever 2n is in the list
 *    (n = 7 uses 16, n = 100 uses 256).  n > 512 gives ORI_ERR_UNSUPPORTED.
 */
#ifndef ORI_H
#define ORI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ori_ctx_s* ori_ctx; /* opaque; owns every device workspace */

typedef enum {
  ORI_OK = 0,
  ORI_ERR_INVALID_ARG = 1,   /* bad size, pointer, value (NaN/Inf, N < 0, ...) */
  ORI_ERR_OUT_OF_MEMORY = 2, /* workspace above the given limit, or hipMalloc failed */
  ORI_ERR_DEVICE = 3,        /* a HIP call failed; the context is poisoned */
  ORI_ERR_BREAKDOWN = 4,     /* COCG breakdown: r^T r = 0 or p^T A p = 0 with r, p != 0 */
  ORI_ERR_NOT_CONVERGED = 5, /* iteration limit reached; u holds the last iterate */
  ORI_ERR_UNSUPPORTED = 6    /* n with no FFT plan */
} ori_status;

typedef enum {
  ORI_FP64 = 0, /* complex128 everywhere */
  ORI_MIXED = 1 /* complex64 FFT matvec, FP64 reductions and FP64 true-residual refinement */
} ori_precision;

typedef enum {
  ORI_OP_SYSTEM = 0,    /* y = x + G0 (D x)            the matrix of eq. 2.19      */
  ORI_OP_SYMMETRIC = 1, /* y = x + S G0 (S x), S^2 = D  its complex-symmetric form */
  ORI_OP_GREEN = 2      /* y = G0 x                     the sum of eq. 3.3.4 alone */
} ori_operator;

/* Bit mask for ori_create: which precisions get workspaces. */
#define ORI_PROVISION_FP64 1
#define ORI_PROVISION_MIXED 2

typedef struct {
  int64_t n;          /* cubes per side (P = n^3 unknowns), n >= 1          */
  double side;        /* edge of the cube domain (> 0); the paper uses 1     */
  double origin[3];   /* corner of the cube domain                           */
  double cell_offset; /* point of each cube: origin + side*(i + offset)/n    */
} ori_grid;

typedef struct {
  double tol;            /* stop when ||r|| / ||b|| < tol (recursive residual of the
                            symmetric system; Section 4's residual-based error)       */
  int32_t max_iter;      /* COCG iteration cap (FP64); total inner iterations (mixed)  */
  int32_t precision;     /* ori_precision                                           */
  int32_t check_every;   /* read the residual norm on the host every this many
                            iterations (>= 1; 0 means 1)                             */
  int32_t use_x0;        /* 1: u holds an initial guess of u on entry                */
  double inner_tol;      /* mixed: relative tolerance of each inner solve (0: 1e-5);
                            an inner solve stops earlier when half of the residual
                            reduction still needed for tol is reached            */
  int32_t max_outer;     /* mixed: refinement cycles (0: 10)                         */
  int32_t true_residual; /* 1: also compute ||u0 - A u|| / ||u0||: one extra
                            matvec, except in mixed precision when u = w / S
                            (no S_p small): there the last FP64 refinement
                            residual r = S (u0 - A u) gives it as ||r / S||  */
  int32_t graph;         /* 1: run each block of check_every COCG iterations as one
                            replay of a HIP graph, built node by node from the
                            same kernels and arguments (no stream capture) and
                            cached per context and precision (the first block,
                            later blocks; up to 8), so results are bitwise those
                            of 0: one launch per kernel.  Safe while other threads use
                            other contexts or the device.  Ignored while
                            per-kernel profiling is enabled.                       */
  int32_t multi;         /* ori_group_solve: 1 runs the COCG iterations of the
                            problems still running in one launch per kernel when
                            every one of them has a padded length in 8..256
                            and the default layout, and neither
                            per-kernel profiling nor the guard checks of
                            ORI_CHECK_GUARDS=1 are on (otherwise, and with 0,
                            each problem launches its own kernels).  The
                            results are bitwise the same either way.  Other
                            calls ignore it.                                    */
} ori_solve_opts;

typedef struct {
  int32_t iterations;       /* COCG iterations (FP64 + inner complex64)            */
  int32_t refinements;      /* mixed: FP64 refinement cycles performed             */
  int64_t matvecs;          /* FFT operator applications, all precisions           */
  int64_t matvecs_c64;      /* ... of which in complex64                           */
  double rel_res_recursive; /* final ||r|| / ||b|| of the symmetric system         */
  double rel_res_true;      /* ||u0 - A u|| / ||u0|| of eq. 2.19, or -1 if not asked */
  double seconds;           /* wall time of the call                               */
} ori_solve_info;

/* Fill opts with the defaults: tol 1e-10, max_iter 1000, FP64, check_every 1,
 * no x0, inner_tol 1e-5, max_outer 10, true_residual 1, graph 1. */
void ori_default_opts(ori_solve_opts* opts);

/* Device bytes of the one workspace block that ori_create takes for this
 * grid, batch size and provision mask (every workspace and its guard band;
 * the twiddle tables of a padded length are shared by all contexts of it).
 * Host-only arithmetic, no device call.  Returns ORI_ERR_INVALID_ARG /
 * ORI_ERR_UNSUPPORTED for a bad grid or batch. */
ori_status ori_workspace_bytes(const ori_grid* g, int32_t nrhs, int32_t provision, int64_t* bytes);

/* Allocate a context and its workspaces for grid g and a batch of nrhs
 * right-hand sides (1 <= nrhs <= 1024) that share one operator (same k, h,
 * N) and differ in the incident field: the coefficient and spectrum
 * buffers, the FFT work arrays and the COCG vectors of every right-hand side.
 * Every per-right-hand-side array of the other calls is then [nrhs][P]
 * (right-hand side i at offset i*P); each product and COCG step runs all of
 * them in the same launches, and the kernel spectrum is read once per pass
 * for the whole batch.  provision: ORI_PROVISION_* mask (FP64 is always
 * provisioned).  mem_limit_bytes > 0 caps the workspace: above it the call
 * returns ORI_ERR_OUT_OF_MEMORY without touching the device.  stream: a
 * hipStream_t (e.g. torch.cuda.current_stream().cuda_stream) or NULL. */
ori_status ori_create(const ori_grid* g, int32_t nrhs, int32_t provision, int64_t mem_limit_bytes,
                      void* stream, ori_ctx* out);

/* Compute the coefficients and the kernel spectrum for wave number k > 0
 * (Sections 2-3): D = 4 pi h N |Delta|, S = sqrt(D), b = S u0, and the FFT
 * of the zero-excluded Green's table G(|m| side/n) on the (2n)^3 grid.
 *   h  : device complex128[P], boundary impedance function h(x_p) (eq. 2.19)
 *   N  : device float64[P], distribution density N(x_p) >= 0 (eq. 2.17);
 *        NULL means N = 1
 *   u0 : device complex128[nrhs][P], incident fields u0(x_p) (eq. 2.4 or any
 *        field), one per right-hand side
 * NaN/Inf anywhere or N < 0 gives ORI_ERR_INVALID_ARG.  May be called again
 * on the same context with new data (no reallocation); the spectrum is then
 * reused while k is unchanged (ori_spectrum_cache). */
ori_status ori_load(ori_ctx ctx, double k, const void* h, const double* N, const void* u0);

/* The kernel spectrum depends only on the grid and k, so ori_load computes
 * it only when k differs from the previous successful load on ctx (design
 * loops that change h or N, or u0, skip it; the results are bitwise those of
 * a fresh computation).  enable = 0 makes every ori_load compute it again
 * (a benchmark that times whole loads); enable = 1 (the default) restores
 * the reuse. */
ori_status ori_spectrum_cache(ori_ctx ctx, int32_t enable);

/* ori_create(g, 1, FP64|MIXED, 0, stream, out) followed by ori_load. */
ori_status ori_setup(const ori_grid* g, double k, const void* h, const double* N,
                     const void* u0, void* stream, ori_ctx* out);

/* Solve eq. 2.19 for u (device complex128[nrhs][P]).  COCG runs on the
 * complex symmetric form (I + S G0 S) w = S u0 and returns u = u0 - G0 S w.
 * A batch runs in lockstep; a right-hand side that has converged stays
 * frozen while the others continue.  opts NULL: defaults.  info (host, may
 * be NULL) receives the worst over the batch (max iterations, max
 * residuals); ori_batch_info gives each right-hand side.  On
 * ORI_ERR_NOT_CONVERGED / ORI_ERR_BREAKDOWN (any right-hand side) u holds the
 * solutions recovered from the last iterates. */
ori_status ori_solve(ori_ctx ctx, const ori_solve_opts* opts, void* u, ori_solve_info* info);

/* Statistics of right-hand side i of the last ori_solve on ctx. */
ori_status ori_batch_info(ori_ctx ctx, int32_t i, ori_solve_info* info);

/* Adjoint of eq. 2.19 for material design.  With u the solution (from
 * ori_solve on this context) and f a device complex128[P] vector, solve
 * A^T lam = f, A^T = I + D G0 (same complex-symmetric COCG, division free:
 * lam = f - S z with (I + S G0 S) z = S G0 f), and return
 *     g_p = -c_p u_p (G0 lam)_p,    c_p = 4 pi N_p |Delta_p|,
 * so that a real functional L(u) with dL = Re sum_j f_j du_j changes by
 * dL = Re sum_p g_p dh_p  (dL/dRe h_p = Re g_p, dL/dIm h_p = -Im g_p) and
 * by dL = Re sum_j lam_j du0_j.  For PyTorch's complex gradient convention,
 * pass f = conj(grad_u); then grad_h = conj(g) and grad_u0 = conj(lam).
 * g, lam: device complex128[P] outputs, either may be NULL (not both).
 * opts: tolerance / precision of the adjoint solve (use_x0 is ignored).
 * Needs a context with nrhs = 1 (else ORI_ERR_UNSUPPORTED). */
ori_status ori_adjoint(ori_ctx ctx, const ori_solve_opts* opts, const void* u, const void* f, void* g, void* lam,
                       ori_solve_info* info);

/* Objective J = sum_j |u_j - t_j|^2 (t = u_target, device complex128[P]):
 * solves eq. 2.19 into u, writes J (host double) and dJdh (device
 * complex128[P]) with dJ = Re sum_p dJdh_p dh_p, i.e. dJ/dRe h_p = Re dJdh_p
 * and dJ/dIm h_p = -Im dJdh_p (the adjoint above with f = 2 conj(u - t)).
 * info sums both solves. */
ori_status ori_gradient(ori_ctx ctx, const ori_solve_opts* opts, const void* u_target, void* u, double* J,
                        void* dJdh, ori_solve_info* info);

/* y = op(x) with the FFT operator (device complex128[nrhs][P] each).
 * precision ORI_MIXED runs the FFT stages in complex64 (inputs and outputs
 * stay complex128).  Used by tests and the benchmark. */
ori_status ori_matvec(ori_ctx ctx, int32_t op, int32_t precision, const void* x, void* y);

/* y = G0 x, the same product as ori_matvec(ctx, ORI_OP_GREEN, precision, x,
 * y) on a context of grid g loaded with wave number k, for callers that
 * cannot allocate device memory: code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc.  No context is needed and nothing
 * is allocated: the kernel spectrum, the twiddle tables and the FFT work
 * arrays live in one static device array of 32 MiB that the library holds
 * on every device it runs on until the process ends, which limits n to 64
 * (larger n give ORI_ERR_UNSUPPORTED with the bytes needed).  x, y: device
 * complex128[P] of the current device (P = n^3), caller owned.  precision:
 * ORI_FP64 or ORI_MIXED (complex64 FFT stages).  Every step -- twiddles,
 * the spectrum of k, the five FFT passes -- is enqueued on `stream` (a
 * hipStream_t, or NULL) with kernel launches only (no memset, copy or
 * synchronization), and the call returns without waiting: y is ready once
 * the stream's work is.  Every call on a device shares that device's
 * array, so calls whose work overlaps on one device (other streams, other
 * threads) race and must be ordered by the caller.  Errors are returned
 * before anything is enqueued; ori_last_error(NULL) gives the text. */
ori_status ori_green_noalloc(const ori_grid* g, double k, int32_t precision, const void* x, void* y,
                             void* stream);

/* ---- several independent problems solved together ------------------------ */

typedef struct ori_group_s* ori_group; /* opaque; owns its problems' workspaces */

/* A group of nprob (1..64) independent problems of eq. 2.19 -- the uneven
 * batch: each its own grid (any n <= 512), wave number, h, N and incident
 * field (one right-hand side), so that no two share an operator.  Allocates
 * what ori_create(&grids[i], 1, provision, 0, ., .) would for each problem,
 * and a stream per problem (so the problems' launches run side by side).
 * stream: the caller's stream (hipStream_t or NULL); every group call starts
 * after the work already queued on it and returns after all of its own work
 * has completed.  Like a context, a group is used by one thread at a time;
 * distinct groups and contexts are independent.  Errors of the ori_group_*
 * calls: ori_last_error(NULL). */
ori_status ori_group_create(const ori_grid* grids, int32_t nprob, int32_t provision, void* stream, ori_group* out);

/* ori_load of problem i (0 <= i < nprob): wave number, h, N, incident field
 * (device arrays of that problem's size, as for ori_load). */
ori_status ori_group_load(ori_group g, int32_t i, double k, const void* h, const double* N, const void* u0);

/* ori_group_load of every problem in one call: k[i], h[i], N[i] (N NULL:
 * all N_i NULL, or N[i] NULL for one problem) and u0[i] for i < nprob, host
 * arrays of device pointers.  Every problem's work is enqueued before the
 * call waits for any of them, so the problems load side by side.  Each
 * problem ends loaded as by ori_group_load; on an error the problems after
 * the failing one are left as they were before the call, or not loaded. */
ori_status ori_group_load_all(ori_group g, const double* k, const void* const* h, const double* const* N,
                              const void* const* u0);

/* Solve every problem (eq. 2.19 by COCG on its complex-symmetric form, as
 * ori_solve).  The problems run in lockstep: each block of check_every
 * COCG iterations of the problems still running is one replay of a HIP
 * graph in which every problem is an independent chain
 * of its own kernels (built node by node, as in ori_solve), so the GPU runs
 * the problems side by side; a problem leaves once it has converged.  Every
 * problem runs exactly the kernels of its own ori_solve, in the same order,
 * so each result is bitwise that of solving the problem alone.
 *   opts: as ori_solve, the same for every problem (NULL: defaults)
 *   u:    host array of nprob pointers, u[i] device complex128[n_i^3]
 *   info: host array of nprob entries, or NULL
 * Returns ORI_OK, or the status of the first problem that did not converge
 * (every u[i] is filled either way). */
ori_status ori_group_solve(ori_group g, const ori_solve_opts* opts, void* const* u, ori_solve_info* info);

/* COCG iterations the group's solves have run in one launch per kernel for
 * all of their problems still running (ori_solve_opts.multi), counted once
 * per iteration of the set, since the group was created. */
ori_status ori_group_multi_iterations(ori_group g, int64_t* iterations);

/* Release the group and its problems' workspaces (NULL is ignored).  Waits
 * for the group's streams; the workspaces and the streams go to the
 * process-wide cache of ori_destroy. */
void ori_group_destroy(ori_group g);

/* ---- what the solution is used for (Section 2, Section 4) ---------------- */

/* Charges of the cells: q_p = -D_p u_p = -c_S h_p N_p |Delta_p| u_p, the sum
 * of the particle charges Q_m = -c_S a^{2-kappa} h(x_m) u_e(x_m) (eq. 2.13)
 * over the a^{-(2-kappa)} N_p |Delta_p| particles of cell p (eq. 2.18).
 * u, q: device complex128[nrhs][P] (u a solution of eq. 2.19 for the loaded
 * data).  Synchronises the context stream. */
ori_status ori_charges(ori_ctx ctx, const void* u, void* q);

/* Scattered field v(x) = sum_p G(x, x_p) q_p at M points (eq. 2.10 with the
 * particles of each cell at x_p, G of eq. 2.6a); u0(x) + v(x) is the total
 * field.  A cell point at distance exactly 0 is left out, as in the sum of
 * eq. 2.19, so at the cell points u0 + v reproduces u.  x: device
 * double[M][3]; v: device complex128[nrhs][M].  Direct sum in FP64, O(M P)
 * work, deterministic.  Synchronises the context stream. */
ori_status ori_scattered_field(ori_ctx ctx, const void* u, const double* x, int64_t M, void* v);

/* Far-field amplitude A(beta) = (1 / 4 pi) sum_p exp(-i k beta . x_p) q_p,
 * so that v(r beta) = A(beta) e^{ikr} / r + O(1/r^2) as r -> infinity.
 * beta: device double[M][3] unit directions; A: device complex128[nrhs][M].
 * Synchronises the context stream. */
ori_status ori_far_field(ori_ctx ctx, const void* u, const double* beta, int64_t M, void* A);

/* Refraction recipe on the grid (P entries each; ctx supplies P, the stream
 * and scratch and need not be loaded).  ori_refraction_index:
 * n = [n0^2 - c_S h N / k^2]^{1/2} (eq. 4.1, from eqs. 2.20a and 2.24) with
 * the branch z^{1/2} = |z|^{1/2} e^{i phi/2}, phi = arg z in [0, 2 pi)
 * (eq. 4.2).  ori_design_impedance: the h that gives n,
 * h = k^2 (n0^2 - n^2) / (c_S N) (eqs. 2.25, 2.26).  c_S: shape constant
 * (4 pi for spheres).  n0, h, n: device complex128[P]; N: device double[P]
 * or NULL for N = 1.  Entries with NaN/Inf, or with N < 0 (N <= 0 for the
 * design), get 0 and make the call return ORI_ERR_INVALID_ARG.
 * Synchronises the context stream. */
ori_status ori_refraction_index(ori_ctx ctx, double k, double c_S, const void* n0, const void* h,
                                const double* N, void* n);
ori_status ori_design_impedance(ori_ctx ctx, double k, double c_S, const void* n0, const void* n,
                                const double* N, void* h);

/* Section 4, the comparison behind Table 4: for solutions x on a fine grid
 * (n_fine per side, points at (i + fine_offset) side / n_fine from the
 * context's origin) and y on the context's grid (the coarse one), the sup
 * over coarse cells Delta_q of the mean of |x_i - y_q| over the fine points
 * inside Delta_q; a fine point lies in cell floor((i + fine_offset) n /
 * n_fine) per axis.  Cells with no fine point are skipped; *diff = -1 if
 * none holds one.  y: device complex128[P]; x_fine: device
 * complex128[n_fine^3]; ctx need not be loaded.  ORI, RED and IE solutions
 * are this solver on nested grids (eqs. 2.15, 2.19, 2.20).  Synchronises
 * the context stream. */
ori_status ori_interpolation_difference(ori_ctx ctx, const void* y, const void* x_fine, int64_t n_fine,
                                       double fine_offset, double* diff);

/* Layout of the FFT passes of one precision.  Performance only: blk_lg and
 * prefetch leave every result bitwise unchanged; narrow tiles and the radix
 * plan may change results at the level of rounding. */
typedef struct {
  int32_t blk_lg;   /* log2 of the row block (along i1) of the work array between
                       the strided and Z passes, 0..6, n divisible by 2^blk_lg  */
  int32_t narrow;   /* 1: narrow pencil tiles (half as many pencils per
                       workgroup) in the two strided passes                     */
  int32_t prefetch; /* 1: the Z pass loads its next tile while it transforms one */
  int32_t znarrow;  /* 1: narrow pencil tiles in the Z pass                      */
  int32_t zplan;    /* radix plan of the Z pass's transforms: 0 the padded
                       length's default, 1 its alternative (another radix
                       order or radices with the same threads per pencil:
                       L = 32, 48, 80, 96, 128, 192, 256, 384, 512, 1024; at
                       L = 1024 it is 16 x 8 x 8, the complex128 default
                       there); 1 is invalid at the other lengths              */
} ori_layout;

/* Layout in use for precision ORI_FP64 (complex128 FFTs) or ORI_MIXED
 * (complex64 FFTs). */
ori_status ori_get_layout(ori_ctx ctx, int32_t precision, ori_layout* out);

/* Set the layout of one precision; ORI_ERR_INVALID_ARG for an invalid one
 * (the layout in use is kept).  Synchronises the context stream. */
ori_status ori_set_layout(ori_ctx ctx, int32_t precision, const ori_layout* layout);

/* Autotuner.  On a loaded context, times the COCG product of each
 * provisioned precision (reps timed products after one warm-up per
 * candidate, reps = 0 means 3) for every valid layout, keeps the fastest on
 * ctx, and records it in a process-wide table keyed by (device, n, nrhs)
 * from which later ori_create calls on that key start.  Overwrites the
 * context's iterate and work vectors (not its loaded data), so call it
 * between solves.  best[2] and ms_per_product[2] (FP64, complex64; either
 * may be NULL) receive the winners and their time per product (-1 for a
 * precision that is not provisioned).  Synchronises the context stream. */
ori_status ori_tune(ori_ctx ctx, int32_t reps, ori_layout* best, double* ms_per_product);

/* Memory-safety check of the library's own workspaces.  Every workspace is
 * followed by a 4 KB guard band of a fixed byte pattern; *damaged receives
 * the number of bands no longer intact (0 unless a kernel wrote past the end
 * of a workspace).  With ORI_CHECK_GUARDS=1 in the environment when a context
 * is created, every kernel launch of that context is followed by this check
 * (graph replay is then off) and a damaged band ends the call with
 * ORI_ERR_DEVICE naming the kernel: a slow debug mode.  Synchronises the
 * context stream. */
ori_status ori_check_guards(ori_ctx ctx, int64_t* damaged);

/* Per-kernel timing with HIP events on the context stream.  enable = 1
 * clears the counters and starts recording every launch; 0 stops. */
ori_status ori_profile_enable(ori_ctx ctx, int32_t enable);

/* Time only the kernel kinds in a comma-separated list of the names that
 * ori_profile_read reports, without their precision suffix ("zpass",
 * "f1,f2", ...); NULL or "" times every kind (the default).  Fewer events
 * cost less inside a timed region.  Unknown names give ORI_ERR_INVALID_ARG
 * and leave the selection as it was. */
ori_status ori_profile_kinds(ori_ctx ctx, const char* kinds);

/* Average device duration (ms) and launch count of each kernel kind since
 * ori_profile_enable(ctx, 1).  names[i] (static strings) identify the kinds;
 * up to max entries are written; *count receives the number of kinds. */
ori_status ori_profile_read(ori_ctx ctx, int32_t max, const char** names, double* avg_ms,
                            int64_t* launches, int32_t* count);

/* Release every device allocation of ctx (NULL is ignored).  Waits for the
 * context's stream.  The workspace (one device block) and the pinned host
 * mirrors (one pinned block) are kept in a process-wide cache, up to 4 GiB
 * of each kind, and a later ori_create or ori_group_create on the same
 * device that needs a block of exactly that size takes it instead of
 * allocating (creating and destroying contexts in a loop then costs no
 * hipMalloc/hipFree); larger blocks are freed at once.  A block taken from
 * the cache holds what its last owner left: nothing in this library reads a
 * workspace before writing it. */
void ori_destroy(ori_ctx ctx);

/* Free every block and stream the process-wide cache holds (ori_destroy,
 * ori_group_destroy), on their devices.  Contexts and groups still alive
 * are not touched.  Safe to call at any time from any thread. */
void ori_release_cached_memory(void);

/* Text of the last error on ctx, or of the last failed ori_create/ori_setup
 * in this thread when ctx is NULL.  Never NULL. */
const char* ori_last_error(ori_ctx ctx);

/* Library version string. */
const char* ori_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ORI_H */
