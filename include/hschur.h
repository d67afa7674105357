/*
 * hschur.h -- C-ABI of the MI355X (gfx950) symmetric near-field
 * Schur-complement preconditioner for ACA-compressed H-matrix solves.
 *
 * The library solves Z x = b with Z complex symmetric (Z = Z^T, Sec. 3.2 of
 * Negi, Balakrishnan & Rao, arXiv 2111.13483), split as Z = Z_N + Z_F
 * (Eq. 11): Z_N the dense leaf-level near field, Z_F the ACA-compressed far
 * field (Eq. 9-10). The preconditioner is the near field scaled to block
 * diagonal form by the symmetric Schur complement (Eq. 12-21), used as
 * P^-1 = alpha D^-1 alpha^T (Eq. 23, 24, 28) inside right-preconditioned
 * GMRES (Eq. 2).
 *
 * Matrix entries are the scalar Helmholtz point kernel
 *   Z_mn = exp(-j k r_mn) / (4 pi r_mn),  Z_mm = (1 - j k h / 2) / (2 pi h).
 *
 * Conventions shared by every entry point
 *  - Complex numbers are interleaved {re, im} doubles (the layout of
 *    torch.complex128); vectors are N x nrhs column-major, leading
 *    dimension N, in the caller's point order.
 *  - Pointers documented "device" must be device memory of the context's
 *    device; "host" pointers are ordinary host memory.
 *  - The caller owns every buffer it passes; the library never frees them
 *    and keeps no pointer to them after the call returns.
 *  - Handles own their device memory, obtained through the context's
 *    allocator callback (hipMalloc when none is given). An hs_precond
 *    refers to its hs_hmatrix, which must outlive it. Handles are
 *    immutable after creation.
 *  - Return value 0 is success, HS_NOT_CONVERGED (1) a warning, negative
 *    values errors. On error every output handle is set to NULL and
 *    hs_last_error() (thread-local) describes the failure.
 *  - Work is enqueued on the context's stream; calls that return results
 *    to the host synchronise that stream before returning.
 */
#ifndef HSCHUR_H
#define HSCHUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define HS_OK               0
#define HS_NOT_CONVERGED    1   /* x holds the best iterate; stats hold true residuals */
#define HS_EINVAL         (-1)  /* bad argument (null pointer, size < 1, duplicate points, ...) */
#define HS_ENOMEM         (-2)  /* device or host allocation failed; earlier handles stay valid */
#define HS_ENODEVICE      (-3)  /* no usable gfx950 device */
#define HS_EHIP           (-4)  /* a HIP runtime call failed */
#define HS_ESINGULAR      (-5)  /* exactly zero pivot in a leaf-block LU */
#define HS_ENUMERIC       (-6)  /* NaN or Inf met, or an ACA rank exceeded its cap */
#define HS_ETIMEOUT       (-7)  /* a device-side wait of the preconditioner apply exceeded the
                                   context's wait limit (hs_context_set_wait_limit); every kernel
                                   still ran to its end, the outputs are unspecified */

/* ---- option enums ------------------------------------------------------ */
#define HS_ORDER_NATURAL    0   /* leaf (octree depth-first) order */
#define HS_ORDER_RCM        1   /* reverse Cuthill-McKee (Algorithm 1, Table 3) */
#define HS_ORDER_CM         2   /* Cuthill-McKee */
#define HS_ORDER_SLOAN      3   /* Sloan's profile and wavefront reduction (Table 3, Fig. 7; used for Sec. 5) */
#define HS_ORDER_KING       4   /* King's front-minimising ordering (Table 3, Fig. 6) */

#define HS_PC_SCHUR         0   /* the symmetric near-field Schur-complement preconditioner */
#define HS_PC_BLOCK_JACOBI  1   /* comparator: P^-1 = blockdiag(Z_kk)^-1, the leaves' own near blocks inverted,
                                   no coupling (ordering and fill_tol ignored; FP64 only) */
#define HS_PC_SCHUR_NONSYM  2   /* comparator (Sec. 3.2, Table 2): the same preconditioner from the non-symmetric
                                   elimination, which keeps both triangles of the working matrix, forms the left
                                   coefficients alpha'_ik = -W_ik W_kk^-1 (Eq. 14) beside the right ones
                                   (Eq. 16) and updates every pair of S_k instead of i <= j; the apply uses
                                   alpha as HS_PC_SCHUR does (alpha' = alpha^T for the symmetric Z here), and
                                   HS_P_ALPHA_LEFT exports alpha' */
#define HS_PC_SCHUR_LOWRANK 3   /* the setup-side low-rank arithmetic (Sec. 3.4 with the cost argument of Sec. 4):
                                   each fill-in block W_kj is compressed (ACA + re-compression at fill_tol) when
                                   step k reaches it, replaced by U V where r (b_k + b_j) < b_k b_j, and carried
                                   in factored form through the coefficient and Schur products; P^-1 is then
                                   exactly (Z_N + Delta)^-1 with Delta_kj = U V - W_kj. One host round trip per
                                   step (the ranks), so it is slower than HS_PC_SCHUR at these leaf sizes;
                                   FP64 only */

#define HS_PREC_FP64        0   /* complex128 throughout */
#define HS_PREC_MIXED       1   /* also keep complex64 copies of the apply's matrices (for HS_SOLVE_FGMRES_MIXED) */

#define HS_SOLVE_GMRES      0   /* right-preconditioned restarted GMRES, FP64 */
#define HS_SOLVE_FGMRES_MIXED 1 /* FP64 flexible GMRES on the FP64 operator; each preconditioning step is an
                                   inner right-preconditioned GMRES on the complex64 operator copies with the
                                   complex64 preconditioner copies (vectors and Arnoldi in FP64); needs
                                   store_c64 at build and HS_PREC_MIXED at setup */
#define HS_SOLVE_TRANSFORMED 2  /* the paper's transformed system (Eq. 25-28): GMRES on
                                   x~ + D^-1 alpha^T Z_F alpha x~ = D^-1 alpha^T b, x = alpha x~ (no near-field
                                   matvec in the iteration); its iteration monitors the transformed residual,
                                   stats report the true ||b - Z x|| / ||b||, which meets tol only up to the
                                   fill-in compression error (alpha^T Z_N alpha = D exactly at fill_tol = 0);
                                   needs P */
#define HS_SOLVE_BLOCK_GMRES 3  /* comparator: coupled block GMRES(restart), one Krylov space shared by the
                                   nrhs columns (block Arnoldi with block CGS2 and Cholesky QR, block
                                   Hessenberg least squares), right-preconditioned by P (NULL = none); iters
                                   counts block steps, max_iters bounds them; at most 256 columns */
#define HS_SOLVE_GMRES_MIXED_IR 4 /* restarted right-preconditioned GMRES whose Arnoldi steps apply the complex64
                                   operator and preconditioner copies (FP32 arithmetic; vectors, Arnoldi and
                                   Givens in FP64), with the true residual recomputed on the FP64 operator at
                                   every restart, so each cycle is one step of iterative refinement; stats and
                                   convergence use that FP64 residual; needs store_c64 and HS_PREC_MIXED like
                                   HS_SOLVE_FGMRES_MIXED */

typedef struct hs_context hs_context;
typedef struct hs_plan    hs_plan;
typedef struct hs_hmatrix hs_hmatrix;
typedef struct hs_precond hs_precond;

typedef void* (*hs_alloc_fn)(size_t bytes, void* user);
typedef void  (*hs_free_fn)(void* ptr, void* user);

typedef struct {
    int32_t leaf_max;     /* octree leaf size: boxes holding more points are split (Sec. 2) */
    double  aca_tol;      /* relative Frobenius tolerance of far-field ACA + re-compression (Eq. 10) */
    int32_t rank_cap;     /* largest ACA rank a far block may reach; 0 = default (256) */
    int32_t store_c64;    /* 1: also keep complex64 copies of the near and far blocks (mixed solves) */
} hs_build_opts;

typedef struct {
    int32_t ordering;     /* HS_ORDER_* (Algorithm 1) */
    double  fill_tol;     /* fill-in compression tolerance (Sec. 3.4); 0 keeps every block dense */
    int32_t precision;    /* HS_PREC_FP64 */
    /* Evaluation layout of the apply (the operator is the same up to rounding):
     * points per chunk of consecutive block rows (0 = 384, at most 384) and
     * columns of the neighbour range folded into each chunk's dense products
     * (0 = 3072; else at least the chunk size, at most 3072). Smaller values
     * send more entries through the pushed far-entry path. */
    int32_t sweep_chunk;
    int32_t sweep_fold_cols;
    int32_t kind;         /* HS_PC_SCHUR (the method), HS_PC_SCHUR_LOWRANK (its setup-side low-rank
                             variant), HS_PC_BLOCK_JACOBI or HS_PC_SCHUR_NONSYM (comparators) */
} hs_precond_opts;

typedef struct {
    int32_t method;       /* HS_SOLVE_GMRES */
    int32_t restart;      /* Krylov dimension m per cycle */
    double  tol;          /* relative residual ||b - Z x|| / ||b|| to reach (Sec. 5 uses 1e-6) */
    int32_t max_iters;    /* cap on inner steps per column; 0 = 5000 */
    int32_t fixed_iters;  /* > 0: run exactly this many inner steps, ignoring tol (parity runs) */
    int32_t inner_steps;  /* HS_SOLVE_FGMRES_MIXED: steps of each inner solve; 0 = 20 */
    double  inner_tol;    /* HS_SOLVE_FGMRES_MIXED: relative tolerance ending an inner solve early; 0 = 1e-2 */
    int32_t use_x0;       /* 1: x holds the initial guess on entry (HS_SOLVE_GMRES only); 0: start from x = 0 */
} hs_solve_opts;

typedef struct {
    int32_t iters;        /* inner GMRES steps taken */
    int32_t converged;    /* 1 if the true relative residual <= tol */
    double  relres;       /* true ||b - Z x|| / ||b|| recomputed at the end */
} hs_solve_stats;

typedef struct {
    int64_t n, nb, nbox, n_near, n_far;
    int64_t n_pattern;      /* off-diagonal blocks of the filled pattern (sum of d_k) */
    int64_t n_fill;         /* of which fill-in blocks (leaves not near) */
    int64_t n_lowrank;      /* fill-in blocks stored as U V */
    int64_t max_dk;         /* largest row of the filled pattern */
    int64_t max_rank;       /* largest far-field rank after re-compression */
    int64_t bytes_near, bytes_far, bytes_alpha, bytes_d;   /* stored matrix bytes */
    int64_t bytes_device;   /* all device memory the handle holds */
    double  flops_setup;    /* algorithmic flops of the Schur elimination (LU + alpha + updates); for an
                               HS_PC_SCHUR_LOWRANK preconditioner, those of its factored arithmetic
                               (compression, coefficients and core products over the compressed panels,
                               expansions) */
    double  flops_fill;     /* ACA/re-compression flops on fill-in blocks, r^2 (m + n) model */
    int64_t bytes_estimate; /* plans only: device bytes an H-matrix plus preconditioner of this plan is
                               expected to hold, computed before any allocation (exact near-field and
                               block-diagonal sizes; far factors at rank min(m, n, 32); three times the
                               dense scaling-coefficient bound for the elimination's working blocks,
                               the stored coefficients and the apply's plan) */
} hs_info;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the default stream). `alloc`/`free` (both or
 * neither) supply device memory; `user` is passed back to them.
 * Errors: HS_ENODEVICE if the device is absent or not gfx950, HS_EINVAL. */
int32_t hs_context_create(hs_context** out, int32_t device, void* hip_stream,
                          hs_alloc_fn alloc, hs_free_fn free_fn, void* user);
/* Change the stream later calls enqueue on. Preconditioner applies (the
 * sweeps of Eq. 23-24 keep workgroups resident and waiting on each other)
 * are ordered library-wide per device: an apply issued on one stream waits
 * for those issued earlier on any other stream, so two never run at once.
 * A stream that has carried applies must stay valid until the context has
 * moved off it (this call or hs_context_destroy). */
int32_t hs_context_set_stream(hs_context* ctx, void* hip_stream);
/* Bound, in seconds, on every device-side wait inside a preconditioner apply
 * (default 5). A wait that polls longer gives up: every kernel of the apply
 * still ends normally, and the call that issued it returns HS_ETIMEOUT.
 * 0 makes a wait give up at its first check unless already satisfied (used
 * by the tests to exercise that path). Errors: HS_EINVAL (NULL, negative). */
int32_t hs_context_set_wait_limit(hs_context* ctx, double seconds);
void    hs_context_destroy(hs_context* ctx);

/* ---- host-only planning: the integer phases ------------------------------
 * Octree (Sec. 2), near/far partition (Eq. 8 with adjacency admissibility),
 * near-field block ordering (Algorithm 1) and the symbolic fill of the
 * scaling coefficients (Sec. 3.3), computed on the host from host points.
 * Needs no GPU; gives exact sizes, footprints and flop counts before any
 * device memory is touched (used for admission by footprint). */
int32_t hs_plan_create(const double* points_xyz_host, int64_t n, int32_t leaf_max,
                       int32_t ordering, hs_plan** out);
int32_t hs_plan_query(const hs_plan* plan, hs_info* info);
void    hs_plan_destroy(hs_plan* plan);

/* Export integer arrays of a plan to host memory (all int64).
 *  HS_X_PERM        N        tree position -> caller index
 *  HS_X_LEAF_OFF    nb+1     tree-order offsets of the leaves
 *  HS_X_BOXES       nbox*7   per box: level, start, count, ax, ay, az, leaf id (-1 if internal)
 *  HS_X_NEAR        n_near*2 leaf pairs (i <= j), sorted
 *  HS_X_FAR         n_far*2  box pairs (t < s in preorder), sorted
 *  HS_X_ORDER       nb       new -> old leaf
 *  HS_X_ROWPTR      nb+1     filled pattern row pointers
 *  HS_X_COLS        n_pattern  column (new index) of each pattern block
 *  HS_X_ORIG        n_pattern  1 if the block pair is a near-field pair, 0 for fill-in
 * `*needed` receives the byte size; with dst == NULL only the size is returned.
 * HS_EINVAL if `cap` is too small. */
#define HS_X_PERM      1
#define HS_X_LEAF_OFF  2
#define HS_X_BOXES     3
#define HS_X_NEAR      4
#define HS_X_FAR       5
#define HS_X_ORDER     6
#define HS_X_ROWPTR    7
#define HS_X_COLS      8
#define HS_X_ORIG      9
int32_t hs_plan_export(const hs_plan* plan, int32_t what, void* dst, int64_t cap, int64_t* needed);

/* ---- H-matrix build (Eq. 9-11) -------------------------------------------
 * points_xyz: device, n x 3 row-major doubles, caller order; copied to the
 * host for the integer phases. k: wavenumber 2 pi / lambda. self_h: spacing
 * h of the self term. Near blocks are assembled on the GPU, far blocks are
 * compressed on the GPU by partial-pivoting ACA then QR + SVD
 * re-compression at opts->aca_tol.
 * The call returns once the near field is assembled (its errors checked);
 * the far field is compressed meanwhile by a library host thread on streams
 * of the H-matrix's own, so the caller's next work (a preconditioner setup,
 * which reads only the near field) runs beside it. Every call that reads
 * the far field (hs_matvec, hs_matvec_noalloc, hs_solve, hs_solve_many, the
 * server, hs_query_hmatrix, hs_hmatrix_export) waits for it first and
 * reports its errors; hs_hmatrix_destroy waits for it too. The context must
 * outlive the H-matrix, as for every object made with it.
 * Errors: HS_EINVAL (n < 1, k < 0, self_h <= 0, leaf_max < 1, coincident
 * points), HS_ENOMEM; from the far field, at the first call that reads it
 * (and every later one): HS_ENOMEM, HS_ENUMERIC (rank above rank_cap). */
int32_t hs_h_build(hs_context* ctx, const double* points_xyz, int64_t n, double k, double self_h,
                   const hs_build_opts* opts, hs_hmatrix** out);
int32_t hs_query_hmatrix(const hs_hmatrix* H, hs_info* info);
void    hs_hmatrix_destroy(hs_hmatrix* H);

/* ---- preconditioner setup (Sec. 3.1-3.4) ---------------------------------
 * Orders the leaf graph, eliminates the near field block row by block on the
 * GPU (LU of W_kk, alpha_kj = -W_kk^-1 W_kj, W_ij += W_ki^T alpha_kj) and
 * compresses fill-in blocks of alpha with ACA + re-compression at
 * opts->fill_tol. Errors: HS_ESINGULAR, HS_ENUMERIC, HS_ENOMEM, HS_EINVAL. */
int32_t hs_precond_setup(hs_context* ctx, const hs_hmatrix* H, const hs_precond_opts* opts,
                         hs_precond** out);
/* Batched setup of count geometries with the same options: the elimination
 * step k of every geometry with more than k leaves runs in one launch per
 * kernel, so many small geometries share launches. out[g] receives the
 * preconditioner of Hs[g]; on error every out[g] is NULL. Results equal
 * those of separate hs_precond_setup calls. */
int32_t hs_precond_setup_many(hs_context* ctx, int64_t count, const hs_hmatrix* const* Hs,
                              const hs_precond_opts* opts, hs_precond** out);
/* Apply-layout autotuner (the evaluation layout of the sweeps, hs_precond_opts
 * sweep_chunk x sweep_fold_cols): sets up H's preconditioner with each layout
 * of a fixed grid (chunks 384, 256, 192 points x folded ranges 3072, 2048,
 * 1536 columns, range >= chunk: 9 layouts), times `reps` applies of nrhs
 * columns of each with HIP events on the context's stream after one warm-up
 * apply, and writes the fastest layout to *best (the other fields as in
 * opts). times_ms (NULL or 9 entries) receives each layout's average apply
 * time in grid order; *ncand (may be NULL) the number of layouts. Every
 * layout gives the same operator (the triangular solves in another order).
 * Errors: HS_EINVAL (NULL, nrhs or reps < 1, a block-Jacobi kind), setup errors. */
int32_t hs_precond_tune(hs_context* ctx, const hs_hmatrix* H, const hs_precond_opts* opts, int32_t nrhs, int32_t reps,
                        hs_precond_opts* best, double* times_ms, int32_t* ncand);
int32_t hs_query_precond(const hs_precond* P, hs_info* info);
void    hs_precond_destroy(hs_precond* P);

/* ---- solve (Eq. 2 with P^-1 of Eq. 23-24, 28) -----------------------------
 * b: device, N x nrhs complex128; x: device, N x nrhs, output (initial guess
 * 0). P may be NULL (unpreconditioned). stats: host array of nrhs entries.
 * Each column is an independent Krylov space; columns share every matrix
 * read. Returns HS_NOT_CONVERGED if some column missed tol. */
int32_t hs_solve(hs_context* ctx, const hs_hmatrix* H, const hs_precond* P,
                 const void* b, void* x, int64_t nrhs, const hs_solve_opts* opts,
                 hs_solve_stats* stats);

/* ---- solves of several geometries at once --------------------------------------
 * Each item is one geometry's system with its own right-hand sides: H, P
 * (NULL = unpreconditioned), b and x device N x nrhs complex128 in the
 * caller's order (x is the initial guess on entry when opts->use_x0). The
 * items' GMRES(m) solves run together: their restart cycles proceed in
 * lockstep, item i's launches on one of up to four streams (item 0 on the
 * context's stream, the others on library streams that first wait for the
 * context's stream), so the work of different geometries overlaps on the
 * device, and one host poll serves all items. Every column is its own Krylov
 * space, so its iterates do not depend on the other columns or items (the
 * same arithmetic as hs_solve up to the rounding order of multi-column
 * kernels). stats: host array of sum(nrhs) entries, item by item. Returns
 * HS_NOT_CONVERGED if some column missed tol. Errors: HS_EINVAL (NULL, bad
 * sizes, a P of another H, a method other than HS_SOLVE_GMRES), HS_ENOMEM,
 * HS_ETIMEOUT, HS_ENUMERIC. */
typedef struct {
    const hs_hmatrix* H;
    const hs_precond* P;
    const void* b;
    void* x;
    int64_t nrhs;
} hs_solve_item;
int32_t hs_solve_many(hs_context* ctx, int64_t nitems, const hs_solve_item* items, const hs_solve_opts* opts,
                      hs_solve_stats* stats);

/* ---- operator applications -------------------------------------------------
 * y = Z_H x (Eq. 11) and z = P^-1 v = alpha D^-1 alpha^T v (Eq. 23-24);
 * device, N x nrhs complex128, caller order. */
int32_t hs_matvec(hs_context* ctx, const hs_hmatrix* H, const void* x, void* y, int64_t nrhs);
int32_t hs_precond_apply(hs_context* ctx, const hs_precond* P, const void* v, void* z, int64_t nrhs);

/* y = Z_H x like hs_matvec, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). The tree-order copies of x and y and the per-block partial
 * results live in a fixed 64 MiB device array of the library (one per
 * device, held until the process ends) instead of memory from the context's
 * allocator: the call allocates nothing and does not synchronise (the result
 * is ready when the context's stream reaches it). The array needs
 * 2 N nrhs + (partial-result slots) nrhs complex128 values, each part rounded
 * up to 256 bytes; *scratch_needed (may be NULL) receives that byte count.
 * Calls that overlap on one device (other streams or threads) share the
 * array and race; issue them in order. Every scratch word read is written
 * in the same call, so nothing needs clearing between calls.
 * Errors: HS_EINVAL (NULL argument, nrhs < 1, more scratch than 64 MiB). */
int32_t hs_matvec_noalloc(hs_context* ctx, const hs_hmatrix* H, const void* x, void* y, int64_t nrhs,
                          int64_t* scratch_needed);

/* ---- kernel timing (measurement) -------------------------------------------
 * Between hs_timing_begin and hs_timing_end every launch of the forward and
 * backward preconditioner sweeps (Eq. 23-24), of the near and far matvec
 * kernels (Eq. 11) and of the two elimination kernels of the setup made
 * through ctx is bracketed by a pair of HIP events on
 * the stream it runs on: ctx's stream, except the near matvec, which runs on
 * the library's second stream beside the far matvec (its time therefore
 * spans the concurrent far kernel). hs_timing_end synchronises ctx's stream
 * (which waits for the second stream after every matvec) and fills out with
 * the launch count and summed event time (ms) per kernel; it resets the
 * record. Intended for benchmarks: the events add a small gap per launch.
 * Errors: HS_EINVAL (NULL argument), HS_EHIP. */
#define HS_KT_SWEEP_FWD 0
#define HS_KT_SWEEP_BWD 1
#define HS_KT_NEAR_MV   2
#define HS_KT_FAR_MV    3
#define HS_KT_FACTOR    4   /* elimination launches holding leaf-block inversions and alpha panel tiles
                               (Eq. 14, 19), with the previous step's Schur tiles beside them when the
                               step takes the look-ahead */
#define HS_KT_SCHUR     5   /* elimination launches of Schur-complement update tiles alone (Eq. 38-42) */
#define HS_KT_ELIM      6   /* a whole elimination (all steps of one setup call) on ctx's stream: its wall
                               time, the launch gaps between its kernels included */
#define HS_KT_COUNT     7
typedef struct hs_kernel_times {
    int64_t launches[HS_KT_COUNT];      /* bracketed (timed) launches */
    double  total_ms[HS_KT_COUNT];      /* summed event time of the bracketed launches */
    int64_t all_launches[HS_KT_COUNT];  /* every launch made while timing was on, bracketed or not */
} hs_kernel_times;
int32_t hs_timing_begin(hs_context* ctx);
/* As hs_timing_begin, but only every `every`-th launch of each kernel
 * (counted from this call, the first one included) is bracketed; every = 1
 * is hs_timing_begin. A sample keeps the events' ordering points out of most
 * of the timed work while the averages stay per launch.
 * Errors: HS_EINVAL (NULL ctx, every < 1). */
int32_t hs_timing_begin_every(hs_context* ctx, int32_t every);
int32_t hs_timing_end(hs_context* ctx, hs_kernel_times* out);

/* ---- test exports (device handles -> host memory) ---------------------------
 * H-matrix:
 *  HS_H_PLAN_*: any HS_X_* code of the plan behind the handle
 *  HS_H_NEAR_OFF   int64 n_near+1  element offsets of the near blocks
 *  HS_H_NEAR_DATA  complex128      near blocks, each b_i x b_j row-major
 *  HS_H_FAR_RANK   int64 n_far     rank after re-compression
 *  HS_H_FAR_OFF    int64 n_far+1   element offsets of the U and V factors
 *  HS_H_FAR_UV     complex128      per far block U (m x r, column-major) then V (r x n, row-major)
 *  HS_H_FAR_PIV    int64 n_far*2*cap ACA pivot log (i, j) per step, -1 padded (cap = rank cap)
 * Preconditioner (blocks indexed by new numbering):
 *  HS_P_D          complex128      D_k = final W_kk, each b_k x b_k row-major
 *  HS_P_ALPHA_KIND int64 n_pattern rank of the stored block, -1 = dense
 *  HS_P_ALPHA_OFF  int64 n_pattern+1 element offsets into HS_P_ALPHA
 *  HS_P_ALPHA      complex128      dense blocks b_k x b_j row-major, or U (b_k x r col-major) then V (r x b_j row-major)
 *  HS_P_ALPHA_LEFT complex128      HS_PC_SCHUR_NONSYM only (else HS_EINVAL): per pattern entry (k, j), in
 *                                  pattern order and back to back, alpha'_jk^T as a dense b_k x b_j row-major
 *                                  block, before fill-in compression
 */
#define HS_H_NEAR_OFF   101
#define HS_H_NEAR_DATA  102
#define HS_H_FAR_RANK   103
#define HS_H_FAR_OFF    104
#define HS_H_FAR_UV     105
#define HS_H_FAR_PIV    106
#define HS_P_D          201
#define HS_P_ALPHA_KIND 202
#define HS_P_ALPHA_OFF  203
#define HS_P_ALPHA      204
#define HS_P_ALPHA_LEFT 205
int32_t hs_hmatrix_export(const hs_hmatrix* H, int32_t what, void* dst, int64_t cap, int64_t* needed);
int32_t hs_precond_export(const hs_precond* P, int32_t what, void* dst, int64_t cap, int64_t* needed);

/* ---- serving ------------------------------------------------------------------
 * Resident geometries on one context (each H-matrix and preconditioner kept in
 * device memory), admitted by device footprint, and continuous batching of
 * right-hand-side columns (Sec. 5 solves each right-hand side on its own; the
 * server shares every matrix read between the columns it runs together).
 * Every geometry has slots_per_geometry column slots of a GMRES(restart)
 * solve. hs_server_step runs one restart cycle of every geometry with live
 * columns, all geometries together (as hs_solve_many). At the cycle boundary
 * finished columns leave their slots (x copied to the request's buffer) and
 * pending requests take free slots, oldest first per geometry, so requests
 * that arrive while others are on the GPU join the running solves without
 * waiting for them to end. A column's iterates do not depend on the others.
 *  hs_server_create: budget in bytes (handles plus the solve workspaces of
 *    their slots), slots_per_geometry in [1, 1024], solve options for every
 *    column (HS_SOLVE_GMRES, use_x0 = 0). The context must outlive the server.
 *  hs_server_add_geometry: host points, build and setup options (popts NULL
 *    = unpreconditioned). The server plans on the host first and refuses with
 *    HS_ENOMEM, before any device allocation, when the plan's footprint
 *    estimate (*estimate, may be NULL) exceeds what is left of the budget;
 *    otherwise it builds the H-matrix and preconditioner (owned by the
 *    server) and charges their actual bytes plus the slots' workspace,
 *    freeing them and refusing with HS_ENOMEM if those exceed the budget.
 *  hs_server_admit: the same for handles the caller built (and keeps alive
 *    until the server is destroyed); an H-matrix shared by several
 *    preconditioners counts once.
 *  hs_server_geometry: the handles of a geometry and the bytes it was charged.
 *  hs_server_submit: b and x device, N x ncols complex128 in the caller's
 *    order (ncols <= slots_per_geometry), owned by the caller until the
 *    request is done; t_arrival on the hs_server_clock() time base (seconds).
 *  hs_server_step: one cycle as above; synchronous; *columns_served = columns
 *    finished in this step (0 when nothing runs). A column that misses tol
 *    within max_iters is not an error: its request's stats say so.
 *  hs_server_pending: requests not yet done and their unfinished columns.
 *  hs_server_request: state of a request (done, iterations, residual,
 *    arrival and completion times). */
typedef struct hs_server hs_server;
typedef struct {
    int32_t geometry;
    int32_t ncols;
    int32_t iters;        /* largest inner-step count over the request's columns */
    int32_t converged;    /* 1 if every column met tol */
    double  relres;       /* largest true relative residual over the columns */
    double  t_arrival;    /* as submitted */
    double  t_done;       /* host clock when its last column had finished */
    int32_t done;
    int32_t pad;
    double  t_start;      /* host clock when its columns took their slots (0 while queued) */
} hs_request_stats;
double  hs_server_clock(void);
int32_t hs_server_create(hs_context* ctx, int64_t device_budget_bytes, int32_t slots_per_geometry,
                         const hs_solve_opts* opts, hs_server** out);
int32_t hs_server_add_geometry(hs_server* s, const double* points_host, int64_t n, double k, double self_h,
                               const hs_build_opts* bopts, const hs_precond_opts* popts, int64_t* estimate,
                               int32_t* geometry);
int32_t hs_server_admit(hs_server* s, const hs_hmatrix* H, const hs_precond* P, int32_t* geometry);
int32_t hs_server_geometry(const hs_server* s, int32_t geometry, const hs_hmatrix** H, const hs_precond** P,
                           int64_t* bytes);
int32_t hs_server_submit(hs_server* s, int32_t geometry, const void* b, void* x, int32_t ncols, double t_arrival,
                         int64_t* request);
int32_t hs_server_step(hs_server* s, int32_t* columns_served);
int32_t hs_server_pending(const hs_server* s, int64_t* requests, int64_t* columns);
int32_t hs_server_request(const hs_server* s, int64_t request, hs_request_stats* out);
void    hs_server_destroy(hs_server* s);

/* ---- errors ----------------------------------------------------------------- */
const char* hs_status_string(int32_t status);
const char* hs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HSCHUR_H */
