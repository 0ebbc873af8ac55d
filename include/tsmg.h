/*
 * tsmg.h — C ABI of the MI355X (gfx950) matrix-free multigrid-preconditioned
 * tensor-product spline smoother of arXiv:1901.00654.
 *
 * The library solves the normal equations of penalised tensor-product
 * B-spline smoothing (Sec. 2.2, eq. 2.4)
 *
 *     (Phi' Phi + lambda Lambda) alpha = Phi' y
 *
 * for scattered data {(x_i, y_i)} in [lo, hi]^d, cubic B-splines (q = 3) on
 * N uniform knot intervals per dimension, without assembling the matrix:
 * Phi'Phi is applied point by point (the Khatri-Rao products of Alg. 3/4) and
 * Lambda through its Kronecker structure (Alg. 2). CG is preconditioned by one
 * geometric multigrid V-cycle (Alg. 7) over the levels g = 1..G,
 * N_g = 2^g (Sec. 3.2.1), with damped Jacobi smoothing (Alg. 6), subdivision
 * prolongation and its transpose (Sec. 3.2.3) and an exact coarse solve on
 * g = 1 (Sec. 3.2.4); the outer loop is Alg. 8.
 *
 * Conventions shared by every call:
 * - Coefficient vectors of level g hold K_g = (N_g + 3)^d entries in C order:
 *   the multi-index (j_1, ..., j_d), 0 <= j_p < N_g + 3, maps to
 *   k = sum_p j_p (N_g + 3)^(d-1-p), j_d contiguous (the "descending
 *   lexicographical order" of Sec. 2.1).
 * - Vector arguments are DEVICE pointers owned by the caller, allocated with
 *   at least the stated length, on the device that was current at ts_create.
 *   Work is enqueued on the problem's stream (ts_options.stream, or a stream
 *   the library creates when that is NULL); calls return once it is enqueued
 *   unless stated otherwise. The caller must not free or modify an argument
 *   before that stream has consumed it.
 * - Every call returns a ts_status. Negative values are errors: the call had
 *   no effect on its outputs beyond what it may have enqueued, and
 *   ts_last_error() gives a message (thread-local, valid until the next
 *   failing call on the same thread). No C++ exception crosses this ABI.
 * - A ts_problem is not thread-safe; distinct problems are independent.
 * - There is one GPU code path per precision and no CPU fallback: if the
 *   device or a kernel is unavailable the call fails with TS_EDEVICE.
 */
#ifndef TSMG_H
#define TSMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ts_problem ts_problem;

typedef enum {
    TS_OK = 0,
    TS_ENOTCONV = 1,      /* iteration limit reached; outputs hold the last iterate */
    TS_EINVAL = -1,       /* an argument is out of range (message says which)       */
    TS_ENOMEM = -2,       /* device allocation failed                               */
    TS_EDEVICE = -3,      /* a HIP runtime call or kernel launch failed             */
    TS_ESINGULAR = -4,    /* the coarse matrix A_c is not positive definite, i.e.
                             an affine function vanishes at every data point and
                             the smoothing problem has no unique solution          */
    TS_EBREAKDOWN = -5    /* CG breakdown: p'Ap <= 0 or a non-finite scalar        */
} ts_status;

typedef enum {
    TS_FP64 = 0,          /* every operation in FP64                                 */
    TS_MIXED_FP32 = 1,    /* PCG whose recurrences, operator applies and V-cycle run
                             in FP32, with FP64 inner products, an FP64 coarse solve
                             and reliable updates: the FP32 correction is added to the
                             FP64 solution and the FP32 residual replaced by the FP64
                             true residual each time it has dropped by inner_tol
                             (iterative refinement that keeps the search direction) */
    TS_MIXED_BF16 = 2,    /* reserved: bfloat16 storage of the per-point 1D basis values
                             of the inner operator; not available in this version
                             (TS_EINVAL)                                              */
    TS_MIXED_FP32_VCYCLE = 3  /* Alg. 8 in FP64 (recurrences, operator applies, inner
                             products) with the V-cycle preconditioner in FP32 on the
                             normalised residual and the flexible (Polak-Ribiere)
                             direction update; iteration counts follow FP64 even
                             where kappa(A) is beyond single precision             */
} ts_precision;

typedef enum {
    TS_PC_MG = 0,         /* one V-cycle (Alg. 7): MGCG, Alg. 8 (default)            */
    TS_PC_NONE = 1,       /* no preconditioner: plain CG on A, the comparison method
                             of Sec. 4 (Table 2 and 3, column CG)                   */
    TS_PC_JACOBI = 2      /* z = D^-1 r with D = diag(A) (Alg. 5 plus the Kronecker
                             diagonal of Lambda)                                    */
} ts_preconditioner;

typedef enum {
    TS_SMOOTH_JACOBI = 0, /* damped Jacobi, Alg. 6 (default)                         */
    TS_SMOOTH_SSOR = 1    /* symmetric successive over-relaxation (Sec. 3.2.2), on
                             the levels whose A_g is assembled as a stencil; levels
                             applied matrix-free keep damped Jacobi. Rows are swept
                             in 4^d colour classes (j_1 mod 4, ..., j_d mod 4) in
                             C order, forward then backward; rows of one class do
                             not couple, so each class is updated at once         */
} ts_smoother;

typedef enum {
    TS_COARSE_DIRECT = 0, /* A_c assembled and inverted once in FP64 (default)       */
    TS_COARSE_CG = 1      /* matrix-free CG on A_c with the diagonal as
                             preconditioner (Sec. 3.2.4), to coarse_tol           */
} ts_coarse_solver;

typedef struct {
    int nu1, nu2;          /* pre/post smoothing steps per level (Alg. 7); default 1, 1 */
    double omega_scale;    /* omega_g = omega_scale / theta_g, theta_g the largest
                              Ritz value of lanczos_steps Lanczos steps on
                              D_g^-1/2 A_g D_g^-1/2 (theta_g <= rho(D^-1 A_g));
                              default 1.8, must be in (0, 2)                       */
    int lanczos_steps;     /* default 16                                             */
    double omega_fixed;    /* > 0: use this omega on every level instead             */
    ts_precision precision;/* used by ts_solve; default TS_FP64                       */
    int max_iter;          /* outer CG iterations (FP64) or total inner iterations
                              (mixed); default 10000                                 */
    double tol;            /* stop when ||b - A alpha||_2 / ||b||_2 <= tol; 1e-8       */
    double inner_tol;      /* mixed: the FP32 residual reduction, since the last FP64
                              update, that triggers the next one; in (0, 1), 0.1      */
    int max_refine;        /* mixed: most FP64 residual updates; default 50          */
    int points_per_block;  /* data-term work per workgroup; 0 = automatic            */
    int stencil_mode;      /* levels whose A_g is assembled at setup as a 7^d-point
                              stencil (same operator, applied as a stencil product):
                              0 = where it is estimated faster and fits (default),
                              1 = none (matrix-free on every level),
                              2 = every level whose stencil fits in memory          */
    void* stream;          /* hipStream_t to enqueue on; NULL = a library stream      */
    int preconditioner;    /* ts_preconditioner; default TS_PC_MG (solve-time)       */
    int smoother;          /* ts_smoother; default TS_SMOOTH_JACOBI (solve-time)    */
    double ssor_omega;     /* SSOR relaxation factor in (0, 2); default 1 (symmetric
                              Gauss-Seidel)                                         */
    int coarse_solver;     /* ts_coarse_solver; default TS_COARSE_DIRECT             */
    double coarse_tol;     /* TS_COARSE_CG: relative residual of the coarse solve;
                              default 1e-14                                         */
    int coarse_max_iter;   /* TS_COARSE_CG: most iterations per coarse solve; 20000 */
    int coarsest_level;    /* c: the V-cycle recurses down to level c and solves A_c
                              there (Sec. 3.2.1, 3.2.4); 1 <= c <= G, default 1; the
                              direct solver needs K_c <= 4096                        */
    const int32_t* degrees;/* NULL, or d B-spline degrees q_p (1..5), one per
                              dimension, replacing ts_create's q (Sec. 2.1); read by
                              ts_create only                                         */
    int deterministic;     /* 1: every result is reproducible bit for bit from run to
                              run on the same device (fixed-order reductions in
                              place of the point pass's LDS and global atomics, and
                              in the setup's moment sums); the point pass takes
                              several times longer (6.4x at d = 3, 2.3x at d = 4 on
                              the benchmark workloads). Cubic splines on equal power-of-two
                              grids only (TS_EINVAL otherwise); read by ts_create
                              only; default 0                                        */
    int bottom_max_k;      /* the V-cycle below the finest level is applied, from the
                              largest level g with K_g <= bottom_max_k (whose A_g
                              is held as a stencil, in the cubic form), by one
                              product with its dense operator B_g (alpha = B_g b,
                              the same linear map as Alg. 7 from g down, assembled
                              at setup); 0 = automatic (2744; 6000 in the general
                              form, whose levels each stream all points), < 0 =
                              never. Used with the damped Jacobi smoother, the
                              direct coarse solver and the nu1, nu2 given to
                              ts_create (other settings run the levels one by
                              one); read by ts_create only                       */
    int vcycle_graph;      /* 1: within ts_solve the V-cycle's kernels are captured
                              once into a HIP graph and replayed each iteration
                              (not on the null stream, nor with the CG coarse
                              solver); 0 (default): launched one by one, which
                              measured 1-2 % faster on MI355X (solve-time)          */
} ts_options;

typedef struct {
    int iterations;        /* CG iterations (FP64 or, mixed, FP32 ones)              */
    int refinements;       /* mixed: FP64 residual updates; FP64: restarts of CG from
                              the true residual                                       */
    int converged;         /* 1 if rel_residual <= tol                                */
    double rel_residual;   /* ||b - A alpha||_2 / ||b||_2 recomputed in FP64 at exit  */
    double setup_s;        /* wall time of ts_create                                 */
    double solve_s;        /* wall time of this ts_solve                             */
    int64_t applies;       /* operator applies (any level, any precision) performed  */
    const double* residual_history;  /* host, history_len entries: the recursive relative
                              residual ||r_k|| / ||b|| before iteration 1 (k = 0) and
                              after each CG iteration (mixed modes: the FP32 one,
                              replaced by the FP64 true residual at each update);
                              owned by the problem, valid until its next ts_solve or
                              ts_destroy                                           */
    int history_len;
} ts_solve_info;

/* Fills *opt with the defaults listed above. */
void ts_default_options(ts_options* opt);

/* Library version string, e.g. "tsmg 0.1 gfx950". */
const char* ts_version(void);

/*
 * Creates a smoothing problem (Sec. 2.2) and runs all setup on the device:
 * bins and sorts the points by knot cell, builds the level hierarchy
 * g = c..G with G = log2(N) and c = opt.coarsest_level (Sec. 3.2.1), the
 * Jacobi diagonals (Alg. 5 plus the Kronecker diagonal of Lambda, Sec. 3.2.2),
 * the damping omega_g, and the coarse solver of level c: A_c and its inverse,
 * or the data of the coarse CG (Sec. 3.2.4).
 *   d          dimension, 1 <= d <= 5
 *   q          spline degree; must be 3
 *   intervals  d ints, knot intervals per dimension; all equal to one power of
 *              two N with 2 <= N and (N + 3)^d < 2^31 and N^d <= 2^30
 *   lo, hi     d doubles (host), the box [lo_p, hi_p], lo_p < hi_p
 *   n          number of points, n >= 1
 *   x          device, n*d doubles, row-major (point i at x[i*d .. i*d+d-1]);
 *              every x must be finite and inside the box
 *   y          device, n doubles, finite
 *   lambda     smoothing weight, finite and > 0
 *   opt        options (NULL = defaults); copied
 *   out        receives the handle
 * x and y are copied into library-owned storage and not retained. Returns
 * TS_EINVAL for bad arguments (including points outside the box or non-finite
 * data), TS_ESINGULAR if A_1 is not positive definite, TS_ENOMEM, TS_EDEVICE.
 * Synchronises the stream before returning.
 */
ts_status ts_create(int d, int q, const int32_t* intervals, const double* lo,
                    const double* hi, int64_t n, const double* x, const double* y,
                    double lambda, const ts_options* opt, ts_problem** out);

/* Releases every resource of the problem (synchronises its stream). NULL is a no-op.
 * Device memory goes back to the library's per-device cache, which later
 * problems draw from; the cache keeps at most min(8 GiB, 1/16 of the
 * device's memory) and is emptied into the device whenever an allocation
 * fails. */
void ts_destroy(ts_problem* p);

/* Replaces the solve-time options of a problem: nu1, nu2, precision, max_iter,
 * tol, inner_tol, max_refine, preconditioner, smoother, ssor_omega, coarse_tol
 * and coarse_max_iter. Setup-time fields (omega_scale, lanczos_steps,
 * omega_fixed, points_per_block, stencil_mode, coarse_solver, coarsest_level,
 * stream) are ignored. Returns TS_EINVAL for negative smoothing counts,
 * tol <= 0, an unknown precision, preconditioner or smoother, or ssor_omega
 * outside (0, 2). */
ts_status ts_set_options(ts_problem* p, const ts_options* opt);

/* Number of levels G (finest level index). */
ts_status ts_num_levels(const ts_problem* p, int* G);

/* K_g = (N_g + 3)^d for level 1 <= g <= G (Sec. 3.2.1). */
ts_status ts_num_coeffs(const ts_problem* p, int level, int64_t* K);

/* The damping omega_g used by the Jacobi smoother on level g (1 <= g <= G; the
 * coarsest level c and the levels below it report 0). */
ts_status ts_get_omega(const ts_problem* p, int level, double* omega);

/* The level g whose V-cycle (Alg. 7 from g down to the coarsest level) is
 * applied as one dense operator under the current options (bottom_max_k of
 * ts_options), or 0 when every level runs its own steps. */
ts_status ts_bottom_level(const ts_problem* p, int* level);

/* b = Phi_G' y on the finest level (Alg. 3; first line of Alg. 8). b: device, K_G doubles. */
ts_status ts_rhs(ts_problem* p, double* b);

/* out = A_g c = (Phi_g'Phi_g + lambda Lambda_g) c (Alg. 4 then Alg. 3, plus Alg. 2 over
 * the Kronecker terms of Lambda, Sec. 2.4), c <= g <= G. c, out: device, K_g doubles,
 * must not alias. */
ts_status ts_apply(ts_problem* p, int level, const double* c, double* out);

/* The same operator evaluated in FP32 arithmetic (the inner operator of the mixed
 * modes; basis values from FP32 cell coordinates). c, out: device, K_g floats. */
ts_status ts_apply_f32(ts_problem* p, int level, const float* c, float* out);

/* D = diag(A_g) (Alg. 5 for Phi_g'Phi_g plus lambda diag(Lambda_g), Sec. 3.2.2),
 * c <= g <= G. D: device, K_g doubles. */
ts_status ts_diag(ts_problem* p, int level, double* D);

/* out = I_{g-1}^{g} e: prolongation from level g-1 to g by the subdivision matrix
 * (eq. 2.6), c < g <= G. e: device K_{g-1} doubles; out: device K_g doubles. */
ts_status ts_prolong(ts_problem* p, int level, const double* e, double* out);

/* out = (I_{g-1}^{g})' r: restriction from level g to g-1 (Sec. 3.2.3), c < g <= G.
 * r: device K_g doubles; out: device K_{g-1} doubles. */
ts_status ts_restrict(ts_problem* p, int level, const double* r, double* out);

/* x = A_c^-1 b on the coarsest level c (Sec. 3.2.4) by the configured coarse solver
 * (TS_COARSE_CG reads residual norms back, so it synchronises the stream every
 * few iterations). b, x: device, K_c doubles. */
ts_status ts_coarse_solve(ts_problem* p, const double* b, double* x);

/* z = one V-cycle (Alg. 7) applied to r from a zero start on the finest level, i.e.
 * the preconditioner of Alg. 8 (FP64). r, z: device, K_G doubles, must not alias. */
ts_status ts_vcycle(ts_problem* p, const double* r, double* z);

/* The same V-cycle in FP32 (coarse solve still in FP64). r, z: device, K_G floats. */
ts_status ts_vcycle_f32(ts_problem* p, const float* r, float* z);

/*
 * Solves (Phi'Phi + lambda Lambda) alpha = Phi'y by Alg. 8 (TS_FP64) or by
 * FP64 iterative refinement around an FP32 Alg. 8 (mixed modes), to the
 * relative FP64 residual opt.tol.
 *   alpha  device, K_G doubles; on entry the start vector when use_start != 0
 *          (else ignored and zero is used); on exit the solution
 *   info   may be NULL
 * Returns TS_OK, TS_ENOTCONV (limit reached, alpha holds the last iterate),
 * TS_EBREAKDOWN, or an error. Synchronises the stream.
 */
ts_status ts_solve(ts_problem* p, double* alpha, int use_start, ts_solve_info* info);

/* yq[i] = s(xq_i) = sum_k alpha_k phi_k(xq_i) (eq. 2.2) at m query points.
 * alpha: device K_G doubles; xq: device m*d doubles row-major; yq: device m doubles.
 * Points outside the box are evaluated on the polynomial piece of the nearest
 * boundary cell. Synchronises the stream. */
ts_status ts_evaluate(ts_problem* p, const double* alpha, int64_t m, const double* xq,
                      double* yq);

/* Measurement of the operator apply A_g c (no effect on the problem's state):
 * enqueues `reps` back-to-back launches of the lambda Lambda_g passes, then
 * `reps` launches of the point pass (Phi_g'Phi_g c, the data-term kernel), on
 * internal vectors filled with a fixed pattern, and reports the average
 * duration of one of each in milliseconds, timed with HIP events recorded on
 * the problem's stream. fp32 != 0 times the FP32 operator. Synchronises. */
ts_status ts_profile_apply(ts_problem* p, int level, int fp32, int reps, double* ms_lambda,
                           double* ms_data);

/* Message of the last failing call on this thread ("" if none). */
const char* ts_last_error(void);

/* Device memory of a problem as allocated by the library: *resident bytes held
 * after setup, *peak the most held at once during setup (sort and stencil
 * temporaries included). Either pointer may be NULL. */
ts_status ts_memory(const ts_problem* p, size_t* resident, size_t* peak);

/* Upper estimate of the peak device bytes a problem of this shape needs from
 * ts_create through ts_solve (the caller's x and y excluded), under the same
 * stencil policy as ts_create. intervals: host, d ints (as for ts_create).
 * opt may be NULL. */
ts_status ts_footprint(int d, int q, const int32_t* intervals, int64_t n, const ts_options* opt,
                       size_t* bytes);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as ts_create + ts_solve from a zero start + ts_destroy, with every
 * device buffer of the problem (sorted points, level hierarchy, stencils,
 * work lists, coarse inverse, Krylov vectors, reduction partials) carved from
 * one static device array of TS_NOALLOC_SCRATCH_BYTES bytes per GPU, which
 * the library holds on each GPU it runs on until the process ends. The call
 * creates no stream, event or pinned host buffer: work runs on opt->stream,
 * or on the null stream when that is NULL, and the call returns after that
 * stream has finished it.
 *   arguments  as for ts_create; alpha: device, K_G doubles, the solution
 *   info       as for ts_solve (may be NULL); residual_history points to
 *              thread-local host memory valid until this thread's next call
 * Returns TS_EINVAL, before any device work, when the problem's estimated
 * peak device memory exceeds the array (and during setup if a buffer does
 * not fit after all), else as ts_create and ts_solve. Calls on one GPU share
 * its array and keep the previous call's contents (every buffer is cleared
 * where the method needs zeros); calls from several threads of a process
 * on the same GPU are serialised by the library, and calls from separate
 * processes do not share an array.
 */
#define TS_NOALLOC_SCRATCH_BYTES (64u << 20)
ts_status ts_solve_noalloc(int d, int q, const int32_t* intervals, const double* lo, const double* hi,
                           int64_t n, const double* x, const double* y, double lambda,
                           const ts_options* opt, double* alpha, ts_solve_info* info);

/*
 * Serving loop: independent smoothing requests (any d, grid, point count, lambda,
 * precision) submitted as they arrive and solved concurrently on one GPU.
 *
 * A server runs `slots` worker threads, each with its own HIP stream. A free
 * worker admits a queued request whose estimated peak device memory
 * (ts_footprint plus its points) fits in what the memory budget has left: by
 * default (TS_ADMIT_SHORTEST) the one that has waited max_wait_s or longer,
 * oldest first, else the one with the least estimated work per operator
 * apply (points x 4^d + coefficients x 7^d), so short requests are not held
 * behind long ones; with TS_ADMIT_FIFO the oldest, which holds back the ones
 * behind it until it fits. The request's points, hierarchy and solver state
 * then live on the device until its solve ends, and the kernels of different
 * requests overlap on the GPU. Each request is solved
 * exactly as ts_create + ts_solve would solve it alone (zero start vector);
 * only the order of floating-point atomic additions differs.
 *
 * Handles are thread-safe: any thread may submit, poll or wait.
 */
typedef struct ts_server ts_server;

typedef enum {
    TS_ADMIT_SHORTEST = 0, /* least estimated work first, overdue requests first (default) */
    TS_ADMIT_FIFO = 1      /* first in, first out                                        */
} ts_admission;

typedef struct {
    size_t memory_budget;  /* bytes of device memory admitted requests may hold at once;
                              0 = half of the free device memory at ts_server_create   */
    int slots;             /* requests solved at once (worker threads); default 4, 1..64 */
    int policy;            /* ts_admission; default TS_ADMIT_SHORTEST                   */
    double max_wait_s;     /* TS_ADMIT_SHORTEST: a request queued this long (seconds)
                              is admitted before shorter ones; default 5               */
} ts_server_options;

typedef struct {
    int d, q;              /* as for ts_create                                        */
    const int32_t* intervals;  /* host, d ints                                        */
    const double* lo;      /* host, d doubles                                         */
    const double* hi;      /* host, d doubles                                         */
    int64_t n;
    const double* x;       /* HOST, n*d doubles row-major; copied by ts_server_submit  */
    const double* y;       /* HOST, n doubles; copied                                  */
    double lambda;
    const ts_options* opt; /* solver options (NULL = defaults); opt->stream is ignored */
} ts_request;

typedef struct {
    ts_status status;      /* outcome of the request's setup and solve                */
    ts_solve_info info;
    int64_t K;             /* number of coefficients of the solution                   */
    size_t footprint;      /* device bytes reserved for it at admission                */
    size_t peak_bytes;     /* device bytes its problem held at most (setup measured)   */
    double t_submit;       /* seconds since ts_server_create: submitted               */
    double t_start;        /* admitted to a worker                                    */
    double t_done;         /* solution copied to host memory                          */
    char error[256];       /* message when status < 0                                 */
} ts_result;

typedef struct {
    int64_t submitted, completed, failed, queued;
    int active;            /* requests on the device now                              */
    int max_active;        /* most requests on the device at once so far              */
    size_t in_use;         /* footprint bytes reserved now                            */
    size_t max_in_use;     /* most footprint bytes reserved at once so far            */
    size_t memory_budget;
} ts_server_stats;

/* Fills *opt with the defaults (memory_budget 0, slots 4, TS_ADMIT_SHORTEST, 5 s). */
void ts_server_default_options(ts_server_options* opt);

/* Starts a server on the current device. Returns TS_EINVAL for slots outside
 * 1..64, an unknown policy or a negative max_wait_s, TS_EDEVICE if no device
 * is usable. */
ts_status ts_server_create(const ts_server_options* opt, ts_server** out);

/* Queues one request and returns at once with its ticket. The host arrays of
 * the request are copied; the caller may reuse them on return. Arguments are
 * checked as far as possible without the device (TS_EINVAL); a request whose
 * footprint exceeds the whole budget is refused with TS_ENOMEM. Errors found
 * later (e.g. points outside the box, a singular A_1) are reported in its
 * ts_result. */
ts_status ts_server_submit(ts_server* s, const ts_request* req, uint64_t* ticket);

/* *done = 1 if the request has finished (successfully or not), else 0. */
ts_status ts_server_poll(ts_server* s, uint64_t ticket, int* done);

/* Blocks until the request has finished, copies its solution (K doubles, C
 * order, finest level) into the HOST buffer alpha when alpha is not NULL,
 * fills *result (may be NULL) and releases the ticket. Any thread may wait,
 * but only one at a time per ticket. Returns TS_EINVAL, without waiting, for
 * an unknown or already released ticket, a ticket another thread is already
 * waiting for, or alpha != NULL with capacity < K; the request's own outcome
 * is result->status. */
ts_status ts_server_wait(ts_server* s, uint64_t ticket, double* alpha, int64_t capacity,
                         ts_result* result);

/* Counters of the server (see ts_server_stats). */
ts_status ts_server_get_stats(ts_server* s, ts_server_stats* stats);

/* Finishes every queued and running request, stops the workers and frees the
 * server (results not yet waited for are discarded). NULL is a no-op. */
void ts_server_destroy(ts_server* s);

#ifdef __cplusplus
}
#endif

#endif /* TSMG_H */
