/*
 * pts.h - C ABI of the space-time BDF1 Newton library for MI355X (gfx950).
 *
 * The library solves the all-at-once BDF1 system of a 2-D scalar conservation
 * law (Section 3, Eq. (4)):
 *     (u^n - u^{n-1}) + tau F(u^n) = 0,   n = 1..N_t,
 * where F is the three-point central discretization of Eq. (3): central
 * differences of the fluxes f = g = cflux u^2 and the conservative viscous
 * operator with face viscosity mu((u_i + u_{i+1})/2), mu(u) = mu_a + mu_b u^2.
 * Each Newton iteration solves the block lower-bidiagonal system of Eq. (6),
 * whose blocks are A_n = I + tau dF/du(u^n) and -I, by the block inverse of
 * Eq. (7) (windows of one level) or the decoupled products of Theorem 1 /
 * Eq. (8) inside windows of W levels.
 *
 * Conventions shared by every entry point
 *   - Arrays are DEVICE pointers owned by the caller, float64, contiguous.
 *     A level is [ny][nx] with x fastest (Section 3, Eq. (4)); the space-time
 *     iterate U is [nt][ny][nx] and holds levels 1..nt; u0 is [ny][nx].
 *   - Dirichlet problems count interior unknowns: node (i, j) sits at
 *     (x0 + (i+1) hx, y0 + (j+1) hy). Periodic problems have nodes
 *     (x0 + i hx, y0 + j hy) and wrap. The library never needs x0, y0.
 *   - Dirichlet data (bdata) is a device array [nt][2(nx+ny)]: per level the
 *     south row (i = 0..nx-1), north row, west column (j = 0..ny-1), east
 *     column. NULL means zero data. Ignored for periodic problems.
 *   - Every call is enqueued on `stream` (NULL = the default stream) and is
 *     asynchronous unless stated otherwise.
 *   - Return value: PTS_OK or a negative PTS_ERR_* code; pts_last_error()
 *     returns a message for the calling thread. No C++ exception crosses the
 *     ABI. On any error the output arrays are left in an unspecified but
 *     finite-or-untouched state, except where stated.
 *   - State the library keeps between calls (all per calling thread, freed at
 *     thread exit): a 4 KiB pinned host buffer for the scalars read back per
 *     Newton step, a pinned staging buffer for batch descriptors and one for
 *     the iteration counts the pipelined multigrid lanes plan (all
 *     hipHostMalloc, grown on demand); up to 32 instantiated HIP graphs of
 *     wavefront sequences (keyed by their launch arguments, oldest dropped);
 *     autotuned plans, stage counts and slab lengths per problem signature,
 *     and each instance's Newton stage count per pipelined batch signature.
 *     pts_autotune additionally allocates one device copy of U for the
 *     duration of the call. Device memory beyond that is the caller's
 *     workspace, except for pts_newton_step_static (see there).
 */
#ifndef PTS_H
#define PTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* pts_stream_t; /* hipStream_t */

enum { PTS_HEAT = 0, PTS_BURGERS = 1 };       /* cflux = 0 | 1/2 (Section 2) */
enum { PTS_DIRICHLET = 0, PTS_PERIODIC = 1 }; /* Eq. (2) | periodic box      */
enum { PTS_FP64 = 0, PTS_MIXED = 1 };         /* inner per-level solve type  */
enum { PTS_SCHED_AUTO = 0, PTS_SCHED_BULK = 1, PTS_SCHED_PIPELINE = 2 };

enum {
  PTS_OK = 0,
  PTS_ERR_INVALID_ARG = -1,   /* bad sizes, NULL pointers, unsupported option */
  PTS_ERR_HIP = -2,           /* a HIP runtime call failed                    */
  PTS_ERR_NONFINITE = -3,     /* NaN/Inf in the input or in a residual        */
  PTS_ERR_SINGULAR = -4,      /* a zero pivot in the banded LU of a level block
                                 (Theorem 1 assumes det A_n != 0)             */
  PTS_ERR_NOT_CONVERGED = -5, /* max_iter reached; U holds the last iterate   */
  PTS_ERR_WORKSPACE = -6,     /* workspace NULL or smaller than required      */
  PTS_ERR_NOT_DOMINANT = -7   /* no level solve with a convergence bound: a
                                 block's Jacobi-scaled Gershgorin radius is
                                 >= 1, or above 0.7 with cell Peclet numbers
                                 above 2 (complex Jacobi spectrum), and the
                                 banded LU does not apply (Dirichlet grids of
                                 at most 64 x 64 nodes)                       */
};

/* One problem instance (Section 2, Eq. (1)-(3)). Read only. */
typedef struct pts_problem {
  int32_t kind;      /* PTS_HEAT or PTS_BURGERS                               */
  int32_t bc;        /* PTS_DIRICHLET or PTS_PERIODIC                         */
  int32_t nx, ny;    /* unknowns per direction, >= 1                          */
  int32_t nt;        /* time levels, >= 1                                     */
  int32_t precision; /* PTS_FP64 or PTS_MIXED (FP32 inner, FP64 refinement)   */
  double hx, hy;     /* grid spacings > 0                                     */
  double dt;         /* uniform step tau > 0 (the paper's runs use uniform tau) */
  double mu_a, mu_b; /* mu(u) = mu_a + mu_b u^2 >= 0                          */
  const double* bdata; /* device [nt][2(nx+ny)] Dirichlet data or NULL       */
  const double* dt_levels; /* device [nt] step sizes tau_n = t^n - t^{n-1} of
                        Eq. (3), each > 0 (not checked), or NULL: dt on every
                        level. With variable steps the solve runs the bulk
                        schedule (Chebyshev or banded level solves); the
                        wavefront schedule, the batched wavefront and
                        multigrid forms, the coarse-grid start and the learned
                        start take uniform steps only (PTS_ERR_INVALID_ARG or
                        the bulk schedule, as stated at each entry point)   */
} pts_problem;

/* Solver options. Zero-initialise for defaults. */
typedef struct pts_options {
  int32_t window;    /* Theorem-1 window W <= 64 (levels decoupled together, Eq. (8)
                        inside each window; runs in the bulk schedule). 0 or 1 =
                        the block inverse of Eq. (7), the stable and cheapest form;
                        pts_window_bound gives the largest W the Section 7
                        condition estimate allows                               */
  int32_t schedule;  /* PTS_SCHED_*: BULK = one Newton iteration after another,
                        replayed as a HIP graph; PIPELINE = Newton iterations
                        overlapped as a wavefront, `stages` of them per
                        sequence (see wave_launch)                             */
  int32_t sweeps;    /* inner Chebyshev sweeps per solve; 0 = from lin_tol     */
  int32_t refine;    /* FP64 refinement passes (PTS_MIXED); < 0 = auto         */
  double lin_tol;    /* relative reduction asked of each per-level solve;
                        0 = 1e-9 (FP64) / 1e-6 per pass (MIXED)                */
  int32_t use_graph; /* BULK only: 1 = capture the iteration in a HIP graph    */
  int32_t stages;    /* PIPELINE only: Newton iterations per launch, 0 = auto  */
  int32_t profile;   /* 1 = time every kernel with HIP events on `stream` (BULK
                        schedule without graph); totals land in pts_stats      */
  int32_t cache_tag; /* solves with different tags keep separate autotuned plans
                        and Newton step counts for the same problem signature
                        (e.g. 1 for starts from a learned initial iterate, 2 for
                        coarse-grid starts, which need fewer steps than the
                        plain one); 0 = default                                 */
  int32_t wave_launch; /* PIPELINE: 0 = one launch per anti-diagonal, replayed
                        from a HIP graph (the faster form on MI355X); 1 = each
                        wavefront sequence as one cooperative launch with a
                        grid barrier between anti-diagonals, when the device
                        holds all its work-groups at once (else as 0)          */
  int32_t barrier_spins; /* PIPELINE, cooperative launch: polls one grid-barrier
                        wait may take before the sequence is abandoned
                        (PTS_ERR_HIP, U left partly updated); 0 = 2^20
                        (about a second)                                       */
} pts_options;

#define PTS_MAX_HIST 64

/* Per-solve statistics, written to HOST memory by pts_solve/pts_newton_step. */
typedef struct pts_stats {
  int32_t iterations;            /* Newton steps applied                       */
  int32_t converged;             /* 1 if ||R||_inf <= tol on exit              */
  int32_t window;                /* W used                                     */
  int32_t sweeps;                /* inner sweeps per solve pass (last step)    */
  int32_t refine;                /* refinement passes per solve (last step)    */
  int32_t schedule;              /* schedule used                              */
  int32_t launches;              /* kernel launches + graph replays issued     */
  int32_t slab;                  /* levels solved all-at-once together: nt, or
                                    the slab length after plain Newton over the
                                    whole domain diverged (see pts_solve)       */
  int32_t hist;                  /* valid entries of the histories below (the
                                    last slab's steps + 1)                      */
  int32_t pad;
  double res_inf[PTS_MAX_HIST];  /* ||R(U_k)||_inf, k = 0..hist-1               */
  double upd_rms[PTS_MAX_HIST];  /* Section 8.1 RMS update norm, k = 1..       */
  double rho_max[PTS_MAX_HIST];  /* max Gershgorin radius of D^-1 A_n at U_k   */
  double solve_ms;               /* wall time inside pts_solve (host clock)    */
  /* filled when pts_options.profile = 1: summed kernel time (ms) and launch count
     per kernel class: [0] residual, [1] per-level solve, [2] update + reductions,
     [3] other (fills, initial iterate). HIP events bracket each launch, except for
     the per-level solves, where they bracket each back-to-back chain (bulk) or
     sequence (wavefront) of launches: time / count is the mean launch interval  */
  double prof_ms[4];
  int32_t prof_count[4];
  /* algorithmic bytes moved by the per-level solve launches of the solve
     (reads of u^n, r^n, du^{n-1}, the iterate of a previous launch; one write)  */
  double level_solve_bytes;
  /* filled by pts_solve_batched with pts_options.profile = 1 on batches whose levels take
     the multigrid-preconditioned solve (every instance's entry holds the batch totals):
     per kernel [0] k_pc_resid, [1] k_mg_down, [2] k_mg_lds, [3] k_mg_up, [4] unused;
     bulk schedule: [5] k_residual, [6] k_update + k_reduce_sum, [7] k_level_absmax;
     pipelined schedule: [5] k_pipe_residual, [6] k_pipe_update, [7] k_pipe_cheb: summed time (ms)
     of the launches, each bracketed by HIP events on `stream`, their number, and their
     algorithmic bytes (the reads and writes the operation needs, once each)          */
  double kern_ms[8];
  int32_t kern_count[8];
  double kern_bytes[8];
} pts_stats;

/* Bytes of device workspace pts_newton_step / pts_solve need for `p`.
   Returns 0 for an invalid problem (see pts_last_error). */
size_t pts_workspace_bytes(const pts_problem* p);

/* Residual and Jacobian blocks at every level (Eq. (5) right-hand side and
   A_n of Eq. (6)).
   U  : device [nt][ny][nx], u0 : device [ny][nx]
   R  : device [nt][ny][nx] output, r^n = -(u^n - u^{n-1} + tau F(u^n))
   coef: device [nt][5][ny][nx] output or NULL; planes C, W, E, S, N hold the
         entries of A_n coupling node (i,j) to itself and to (i-1,j), (i+1,j),
         (i,j-1), (i,j+1) (wrapped when periodic; 0 for a Dirichlet boundary
         neighbour).
   res_inf: device double[1] output or NULL, max |R|. */
int pts_assemble(const pts_problem* p, const double* U, const double* u0, double* R,
                 double* coef, double* res_inf, pts_stream_t stream);

/* One all-at-once Newton step U <- U + dU, dU = M^{-1} R (Eq. (6)) computed by
   the block inverse (Eq. (7)) / Theorem 1 windows with inexact per-level solves
   of relative accuracy opts->lin_tol. Synchronises the stream once to read
   ||R||_inf. stats (host, may be NULL) receives res_inf[0] = ||R(U_in)||. */
int pts_newton_step(const pts_problem* p, double* U, const double* u0, void* workspace,
                    size_t workspace_bytes, const pts_options* opts, pts_stats* stats,
                    pts_stream_t stream);

/* pts_newton_step without a caller workspace and without any allocation: for callers
   that cannot allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid hipMalloc). It computes the same step as
   pts_newton_step in the bulk schedule (the same kernels, so the same result), with
   its scratch in a device array of the library, one per GPU, 64 MiB, reserved when
   the library is loaded on that GPU and held until the process ends. No hipMalloc,
   hipHostMalloc, hipFree, event or graph creation, and no host heap allocation; the
   scalars read back per step go through a stack buffer.
   Limits: problems whose pts_workspace_bytes exceed 64 MiB (about 2.5 M space-time
   nodes) are rejected with PTS_ERR_WORKSPACE before any device work;
   opts->profile = 1 is rejected (PTS_ERR_INVALID_ARG). The calling thread's current
   device must be the device of U, u0 and stream.
   Every call on one GPU uses that GPU's one scratch array, which keeps the previous
   call's contents (nothing in it needs to start at zero): calls that overlap on one
   GPU (other threads, other streams) race and must be serialised by the caller.
   Synchronises the stream once, as pts_newton_step does. */
int pts_newton_step_static(const pts_problem* p, double* U, const double* u0, const pts_options* opts,
                           pts_stats* stats, pts_stream_t stream);

/* Theorem 1 in the paper's own form (Section 4, Eq. (8); Section 5, Eq. (9) and
   Algorithm 1): one Newton step whose levels are decoupled through the explicit
   products P^l = A_1 A_2 ... A_l (P^1 = A_1, P^l = P^{l-1} A_l) and right-hand
   sides rt^l = P^{l-1} r^l + rt^{l-1} (rt^1 = r^1), every level then solving
   P^l du^l = rt^l on its own: rows of P^l and rt^l divided by P^l's diagonal
   (the Section 7 diagonal preconditioner), banded LU without pivoting (the
   paper's direct solver for banded matrices; half-bandwidth min(l nx, nx ny - 1)
   in the x-fastest ordering). P^l is held as the 2 l^2 + 2 l + 1 diagonals of the
   Section 5 remark. In exact arithmetic the step equals the block inverse of
   Eq. (7); in floating point the products' condition numbers grow like K^l
   (Section 7, Eq. (cond)), so the form is meant for the paper's own small
   workloads (pts_window_bound estimates the safe number of levels).
   Dirichlet problems only (PTS_ERR_INVALID_ARG otherwise). Workspace:
   pts_products_workspace_bytes(p) bytes, 256-byte aligned (it grows like
   nx^2 ny nt^2: 2.1 GB at 63 x 63 x 32). Zero or non-finite pivots:
   PTS_ERR_SINGULAR. stats (host, may be NULL): res_inf[0] = max |R(U_in)|,
   upd_rms[1] the RMS update. Synchronises the stream once. */
size_t pts_products_workspace_bytes(const pts_problem* p);
int pts_newton_step_products(const pts_problem* p, double* U, const double* u0, void* workspace,
                             size_t workspace_bytes, pts_stats* stats, pts_stream_t stream);

/* The Newton iteration of pts_solve with every step taken by pts_newton_step_products,
   until max |R| <= tol or max_iter steps (stats->res_inf / upd_rms: the histories). */
int pts_solve_products(const pts_problem* p, double* U, const double* u0, double tol, int max_iter,
                       void* workspace, size_t workspace_bytes, pts_stats* stats, pts_stream_t stream);

/* The product P^n (1 <= n <= nt) of the blocks A_1 .. A_n at the iterate U, in the
   diamond storage of pts_newton_step_products: out is a device array
   [2n^2 + 2n + 1][ny][nx], entry e of node (x, y) coupling it to node (x + b, y + a),
   the entries ordered by a = -n..n, then b = -(n - |a|)..(n - |a|) (0 where that node
   lies outside the grid). Workspace as pts_newton_step_products. */
int pts_product_diamond(const pts_problem* p, const double* U, const double* u0, int n, double* out,
                        void* workspace, size_t workspace_bytes, pts_stream_t stream);

/* Initial space-time iterate of plain Newton: u^n = u^0 for n = 1..nt. */
int pts_init_plain(const pts_problem* p, double* U, const double* u0, pts_stream_t stream);

/* Newton iteration from the iterate in U until ||R(U)||_inf <= tol (tau-scaled,
   absolute, all levels) or max_iter steps. U is overwritten with the result;
   on PTS_ERR_NOT_CONVERGED it holds the last iterate so a later call resumes.
   Safeguard: if the Newton iteration over the whole domain diverges (non-finite or
   exploding residual), the levels are solved in consecutive slabs of L levels, each
   all-at-once from the plain iterate of its own initial level, L halved until every
   slab converges; the root is unchanged. The working L is remembered per problem
   and reported in stats->slab; iterations then counts the steps of all slabs.
   Synchronises the stream (once per Newton step, or per launch when
   pipelined). */
int pts_solve(const pts_problem* p, double* U, const double* u0, double tol, int max_iter,
              void* workspace, size_t workspace_bytes, const pts_options* opts,
              pts_stats* stats, pts_stream_t stream);

/* Autotuner of the wavefront schedule: tries inner sweep/pass plans on this problem
   (each a full solve from the iterate in U, timed with HIP events on `stream`), and
   keeps the fastest converging plan with its Newton step count in a per-thread cache
   keyed by the problem and tol; later pts_solve calls with default options use it.
   U is restored before returning. stats (host, may be NULL) receives the chosen plan
   (sweeps, refine, iterations) and its time in solve_ms. Synchronises the stream. */
int pts_autotune(const pts_problem* p, double* U, const double* u0, double tol, int max_iter,
                 void* workspace, size_t workspace_bytes, const pts_options* opts,
                 pts_stats* stats, pts_stream_t stream);

/* Independent instances (Theorem 1 per instance) solved together.
   Instances of one problem (equal kind, bc, sizes, spacings, dt, mu_a, mu_b,
   precision and bdata pointer; only u0 and the starting iterate differ) run
   batched wavefront sequences unless opts asks for the bulk schedule, windows
   or the cooperative launch (with opts->profile = 1 every sequence is bracketed
   by HIP events: stats prof_ms[1] / prof_count[1] = mean launch interval of the
   wavefront kernel, level_solve_bytes its algorithmic bytes): each anti-diagonal of a sequence is one
   launch over (stages x tiles, instances), all instances run the same stage
   count, and an instance leaves the batch when max|R| <= tol (stats report
   schedule PTS_SCHED_PIPELINE). An instance whose Newton iteration turns
   non-finite or loses diagonal dominance is then solved alone as pts_solve does
   (slabs from the plain iterate). If the inner solve does not fit the wavefront
   kernel the batch takes the bulk schedule (PIPELINE asked: PTS_ERR_INVALID_ARG).
   Otherwise (sizes, level counts and inner plans may differ) every Newton step
   runs the level solves of all instances that have level n in shared launches
   (bulk schedule, work items sorted by level count, per-instance descriptors in
   the workspace header).
   Batches of Dirichlet heat on square grids with h_x = h_y and mu_a > 0 whose
   blocks are stiff (Jacobi Gershgorin radius >= 0.97) solve each level with
   Chebyshev iteration preconditioned by I + tau mu_a (-Delta_h), applied
   approximately by one geometric multigrid V-cycle in float32 (residuals and
   updates in float64; inexact, residual reduced 1e3-fold per level solve unless
   opts->lin_tol says otherwise). Unless opts->schedule is PTS_SCHED_BULK (one
   Newton step at a time), such a batch runs opts->stages Newton steps (default
   and at most 7) per pass over the diagonals D = n + s: Newton stage s works on
   level n at diagonal D, every stage of every instance with its own level
   solver ("lane", in the workspace header), the launches of a diagonal
   carrying all lanes that have a level there; after each pass the residual of
   the result decides which instances run another pass (stats: schedule
   PTS_SCHED_PIPELINE, iterations a multiple of the stage count, res_inf and
   rho_max of the steps inside a pass from the stage residuals the lanes formed,
   upd_rms NaN). Without opts->stages, a batch solved again with the same
   signature (kinds, sizes, coefficients, precision, tol, opts->cache_tag) gives
   each instance the Newton steps it needed before (the largest count seen; in
   as many passes of at most 7 stages as the largest needs; a pass that falls
   short is followed by passes of 2 stages; a per-thread cache). This path
   synchronises the stream once per diagonal (it reads back the iteration
   counts the lanes planned). Instances with different
   boundary kinds or precisions, opts->schedule = PTS_SCHED_PIPELINE (for
   instances that are not one problem) or opts->window > 1 are solved one after
   another with pts_solve.
   U[i], u0[i] are device pointers; workspace is one 256-byte aligned block of
   pts_workspace_bytes_batched bytes; stats is a host array of nprob entries
   (may be NULL). Every instance is attempted; the return code is the first
   error met (pts_last_error names the instance), converged instances hold their
   solutions, failed ones their last iterate. Synchronises the stream once per
   Newton step (bulk) or per wavefront sequence (batched wavefront). */
size_t pts_workspace_bytes_batched(const pts_problem* probs, int nprob);
int pts_solve_batched(const pts_problem* probs, int nprob, double* const* U,
                      const double* const* u0, double tol, int max_iter, void* workspace,
                      size_t workspace_bytes, const pts_options* opts, pts_stats* stats,
                      pts_stream_t stream);

/* Autotuner of the batched wavefront schedule, for instances of one problem (as
   pts_solve_batched defines it; PTS_ERR_INVALID_ARG otherwise): tries inner
   sweep/pass plans on the whole batch (each a full batched solve from the
   iterates in U, timed with HIP events on `stream`) and keeps the fastest
   converging plan with its Newton step count in a per-thread cache keyed by the
   problem, tol and opts->cache_tag, used by later pts_solve_batched calls on
   such batches (a batch is throughput-bound where one instance is
   latency-bound, so its best plan differs from the one pts_autotune keeps for
   pts_solve). U is restored before returning. Arguments as pts_solve_batched;
   stats (host array of nprob entries, may be NULL) receive the chosen plan and
   its time in solve_ms. Synchronises the stream. */
int pts_autotune_batched(const pts_problem* probs, int nprob, double* const* U,
                         const double* const* u0, double tol, int max_iter, void* workspace,
                         size_t workspace_bytes, const pts_options* opts, pts_stats* stats,
                         pts_stream_t stream);

/* Section 4: the paper's initial iterate. The problem is solved on a grid coarsened
   by cf in each spatial direction and in time, and the coarse solution is carried to
   the fine space-time grid by 1-D cubic splines.
   Coarse grid: where cf divides nx (periodic) or nx + 1 (Dirichlet; likewise ny),
   node k is fine node k cf (periodic) or fine interior node (k+1) cf - 1 (Dirichlet:
   the domain edges stay); otherwise the coarse grid spans the same domain with nx / cf
   (periodic) or (nx + 1) / cf - 1 (Dirichlet) evenly spaced nodes. ceil(nt / cf)
   coarse levels of step cf dt (coarse level m at t = m cf dt; the last may lie past the
   fine end time). u0 at a coarse node: the bilinear interpolant of the fine u0 (the
   fine value where the node is a fine node); Dirichlet data by injection (coarse level
   m takes fine level m cf; these need cf to divide nx + 1, ny + 1 and nt). Solved in
   FP64 by the all-at-once Newton iteration from its plain iterate (by Theorem 1 the
   root is the sequential coarse solution) to max|R| <= tol within max_iter steps.
   Splines: along x, then y (periodic lines closed with the period; Dirichlet lines
   through the edge values, coarse west/east data for x lines and fine south/north
   data for y lines, not-a-knot end conditions), then along t through u0 (t = 0) and
   the coarse levels, not-a-knot end conditions, evaluated at every fine node and level.
   Requirements: cf >= 2 leaving >= 3 coarse nodes per periodic axis or >= 1 per
   Dirichlet axis, uniform steps (dt_levels NULL); otherwise PTS_ERR_INVALID_ARG
   (pts_coarse_workspace_bytes then returns 0).
   u0: device [ny][nx]; U: device [nt][ny][nx], written; workspace: device, 256-byte
   aligned, pts_coarse_workspace_bytes(p, cf) bytes; stats (host, may be NULL): the
   coarse solve's statistics. An error of the coarse solve is returned as it is (U is
   then not written). Synchronises the stream. */
size_t pts_coarse_workspace_bytes(const pts_problem* p, int cf);
int pts_coarse_initial_iterate(const pts_problem* p, int cf, const double* u0, double* U,
                               double tol, int max_iter, void* workspace,
                               size_t workspace_bytes, pts_stats* stats, pts_stream_t stream);

/* The coarse-grid start of nprob instances, instance i described by probs[i] (grids
   and level counts may differ; kind and boundary kind are shared), with u0[i] and
   U[i] device arrays: the coarse problems share batched launches (pts_solve_batched),
   then each instance's splines run. workspace: pts_coarse_workspace_bytes_batched(probs,
   nprob, cf) bytes, 256-byte aligned; stats: host array of nprob entries or NULL.
   Errors as pts_coarse_initial_iterate (an instance's coarse solve error is returned as
   pts_solve_batched returns it). */
size_t pts_coarse_workspace_bytes_batched(const pts_problem* probs, int nprob, int cf);
int pts_coarse_initial_iterate_batched(const pts_problem* probs, int nprob, int cf,
                                       const double* const* u0, double* const* U, double tol,
                                       int max_iter, void* workspace, size_t workspace_bytes,
                                       pts_stats* stats, pts_stream_t stream);

/* Section 7, Eq. (cond): largest number of levels W whose product of blocks
   keeps the estimated condition number K^W below c h^4 / eps, with
   K = (1 + 8 mu tau/h^2)/(1 + 2 pi^2 mu tau). If tau <= 0 the paper's setting
   tau = 1/W is used (the worked example N_x = 64, mu = 1e-3, c = 1,
   eps = 1e-16 gives 22). Host function, no device work. */
int pts_window_bound(double h, double mu, double tau, double c, double eps, int wmax);

/* Thread-local message describing the last error (never NULL). */
const char* pts_last_error(void);

/* Library version string. */
const char* pts_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PTS_H */
