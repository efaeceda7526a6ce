/*
 * invaskit.h -- C ABI of the MI355X (gfx950) INV-ASKIT factor/solve library.
 *
 * The library factors A = lambda*I + K~ and solves A x = b, where K~ is the
 * ASKIT hierarchical (HODLR-type) approximation of a Gaussian kernel matrix
 * (Yu, March, Xiao, Biros, "INV-ASKIT: A Parallel Fast Direct Solver for
 * Kernel Matrices", Section II).  The tree, skeletons and interpolation
 * matrices P are inputs, produced by a separate setup step.
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status: INVASKIT_OK (0) or a negative
 *    INVASKIT_E_* code.  Nothing throws or aborts across the ABI.  The text
 *    of the last error is available from invaskit_last_error().
 *  - "DEVICE" pointers are HIP device memory on the current device; "HOST"
 *    pointers are ordinary host memory.  Matrices are column-major unless
 *    stated otherwise; all point and vector data is in tree order (the order
 *    in which every tree node owns a contiguous range).
 *  - Nodes use heap numbering: root 0, children of node i are 2i+1 (left)
 *    and 2i+2 (right); level k holds nodes 2^k-1 .. 2^(k+1)-2; every leaf is
 *    at level `depth`.
 *  - All GPU work is enqueued on the stream given to invaskit_factor(); the
 *    calls that must read results back (factor: pivot status; solve: refine
 *    residuals) synchronize that stream before returning.
 *  - One handle may be used by one host thread at a time.
 *  - The library allocates no device memory.  The caller allocates a
 *    factorization's workspace (size: invaskit_factor_workspace_bytes) and
 *    a solve's or product's scratch (invaskit_solve_workspace_bytes,
 *    invaskit_matvec_workspace_bytes), all DEVICE, 256-byte aligned, and
 *    frees them after the handle is destroyed.  A workspace or scratch that
 *    is too small fails with INVASKIT_E_WORKSPACE before any launch.  A
 *    handle holds one small pinned HOST buffer (hipHostMalloc, freed by
 *    invaskit_destroy) into which the pivot status and the refinement's
 *    column norms are copied back with the stream.
 */
#ifndef INVASKIT_H
#define INVASKIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define INVASKIT_OK               0
#define INVASKIT_E_ARG           -1 /* invalid argument; nothing was launched  */
#define INVASKIT_E_WORKSPACE     -2 /* workspace or scratch too small; nothing
                                       was launched                            */
#define INVASKIT_E_HIP           -3 /* a HIP runtime call failed               */
#define INVASKIT_E_SINGULAR      -4 /* zero or non-finite pivot (node named)   */
#define INVASKIT_E_NOT_CONVERGED -5 /* refinement stalled or hit its cap       */
#define INVASKIT_E_DEVICE        -6 /* no usable gfx950 device                 */

/* element types */
#define INVASKIT_F64 0
#define INVASKIT_F32 1

/* precision modes */
#define INVASKIT_PREC_FP64  0 /* every step in FP64                               */
#define INVASKIT_PREC_MIXED 1 /* FP32 factors, FP64 top-level reduced systems,
                                 FP64 residuals and updates, iterative refinement */

/*
 * Problem description (Section II-B, II-C).  N points in d dimensions,
 * ordered by a complete binary tree of depth L with 2^L leaves.
 *
 *  points        DEVICE, n x d row-major, element type points_dtype.
 *                Borrowed: must stay valid and unchanged until
 *                invaskit_destroy(), because solve/matvec re-read it.
 *  leaf_offsets  HOST, 2^L + 1 entries: leaf j owns points
 *                [leaf_offsets[j], leaf_offsets[j+1]); [0] = 0, last = n,
 *                every leaf non-empty and at most 1024 points.  Copied.
 *  skel_offsets  HOST, 2^(L+1) entries (n_nodes + 1): node c's skeleton is
 *                skel_index[skel_offsets[c] .. skel_offsets[c+1]).  The root
 *                has none; every other node has 1..512 skeleton points.
 *                Copied.
 *  skel_index    HOST, tree-order point ids.  A leaf's skeleton lies in the
 *                leaf; an internal node's skeleton is a subset of its
 *                children's skeletons (nested skeletons).  HOST because the
 *                nesting is checked before any launch; copied into the
 *                workspace.
 *  p_offsets     HOST, n_nodes + 1 entries into p_values.  Copied.
 *  p_values      DEVICE, FP64.  Leaf c: P_{c~ c}, s_c x |c| row-major, columns
 *                in the leaf's point order.  Internal c: P_{c~ [l~ r~]},
 *                s_c x (s_l + s_r) row-major, columns [l~ | r~].  Borrowed
 *                like `points`.
 *  h             Gaussian bandwidth, K(x,y) = exp(-|x-y|^2 / (2 h^2)).
 */
typedef struct invaskit_problem {
  int64_t n;
  int32_t d;
  int32_t depth;
  int32_t points_dtype; /* INVASKIT_F64 or INVASKIT_F32 */
  int32_t reserved0;
  const void* points;
  const int64_t* leaf_offsets;
  const int64_t* skel_offsets;
  const int32_t* skel_index;
  const int64_t* p_offsets;
  const double* p_values;
  double h;
} invaskit_problem;

/*
 * Refinement modes (invaskit_options.refine).  Every mode measures residuals
 * r = b - (lambda*I + K~) x with the FP64 hierarchical product
 * (invaskit_matvec) and updates x in FP64; the factors (FP32 in mixed mode,
 * FP64 in FP64 mode) serve as the approximate inverse M^-1.
 *  AUTO   iterative refinement x += M^-1 r while every step at least halves
 *         the worst column's residual; if a step does not, restarted
 *         flexible GMRES on A, right-preconditioned by M^-1, continues from
 *         the best iterate (GMRES-based refinement: it converges in cases
 *         where M^-1 is too inaccurate for plain refinement, e.g. FP32
 *         factors of an ill-conditioned lambda*I + K~).  In FP64 mode the
 *         first step is the direct solve, so a well-conditioned problem
 *         costs one solve and one product.
 *  IR     iterative refinement only; stops on convergence, at the cap, or
 *         when the residual has not halved over three iterations.
 *  GMRES  restarted flexible GMRES from x = 0.
 *  NONE   one direct solve, no refinement.  The residual is computed (one
 *         product) only when info is requested; then a residual above
 *         refine_tol returns INVASKIT_E_NOT_CONVERGED like the other modes.
 */
#define INVASKIT_REFINE_AUTO  0
#define INVASKIT_REFINE_IR    1
#define INVASKIT_REFINE_GMRES 2
#define INVASKIT_REFINE_NONE  3

typedef struct invaskit_options {
  int32_t precision;        /* INVASKIT_PREC_FP64 (default) or _MIXED            */
  int32_t fp64_top_levels;  /* mixed mode: reduced systems at levels < this are
                               factored in FP64 (default 4)                       */
  double refine_tol;        /* stop when |b - A x|_2 / |b|_2 <= tol for every
                               column (default 1e-10)                             */
  int32_t max_refine_iters; /* cap on refinement steps x += M^-1 r, the first
                               (direct) solve included (default 30)              */
  int32_t tune;             /* INVASKIT_TUNE_AUTO (default) or _OFF, see below   */
  int32_t leaf_lu_panel;    /* 0 (default): per `tune`; 16 or 32: LU panel width
                               of the leaf blocks                                 */
  int32_t leaf_trsm_cols;   /* 0 (default): per `tune`; 16 or 32: right-hand
                               sides per workgroup in the leaf solves of the
                               factorization                                      */
  int32_t leaf_lu_waves;    /* 0 (default): per `tune`; 4 or 8: waves (of 64
                               lanes) per matrix in the leaf LU                   */
  int32_t refine;           /* INVASKIT_REFINE_* (default AUTO)                   */
  int32_t gmres_restart;    /* Krylov vectors per GMRES cycle, 2..64 (default 20) */
  int32_t max_gmres_iters;  /* cap on GMRES steps over all cycles (default 300)  */
  int32_t lambda_group;     /* invaskit_factor_sweep: lambdas per batched launch
                               (0, the default: all of them)                      */
  int32_t zlu_form;         /* 0 (default): per `tune`; INVASKIT_ZLU_ONE_WAVE or
                               INVASKIT_ZLU_BLOCK: the LU form of the reduced
                               systems of order up to 192 on every level          */
  int32_t zsolve_cols;      /* 0 (default): per `tune`; 16 or 32: right-hand sides
                               per workgroup in the sweep's reduced-system solves */
  int32_t leaf_pivoting;    /* INVASKIT_LEAF_PIVOT_AUTO (default) or _PARTIAL,
                               see below                                          */
} invaskit_options;
#define INVASKIT_ZLU_ONE_WAVE 1
#define INVASKIT_ZLU_BLOCK    2

/*
 * Leaf factorization.  The leaf blocks lambda*I + K_aa of Algorithm 1 are
 * symmetric, and positive definite when lambda > 0 (the Gaussian kernel
 * matrix is positive semidefinite): a symmetry the paper leaves unexploited
 * (Section I, limitations).  For such matrices LU without row exchanges is
 * backward stable (its pivots are the positive diagonal of the LDL^T
 * factorization), and dropping the pivot search takes the per-column
 * reduction and barrier out of the leaf LU's panel.
 *  INVASKIT_LEAF_PIVOT_AUTO     when lambda > 0 (every lambda of a batched
 *                               sweep group), the leaf blocks of orders above
 *                               the one-wave limit are factored without row
 *                               exchanges; if a pivot comes out not positive
 *                               and finite (a block not numerically positive
 *                               definite, e.g. a tiny lambda in FP32), the
 *                               whole factorization runs again with partial
 *                               pivoting.  With lambda <= 0, partial pivoting.
 *  INVASKIT_LEAF_PIVOT_PARTIAL  always partial pivoting (LAPACK getrf).
 * Either way the factors have the layout the solves read (a permutation,
 * the identity without row exchanges, and packed L\U).
 */
#define INVASKIT_LEAF_PIVOT_AUTO    0
#define INVASKIT_LEAF_PIVOT_PARTIAL 1

/*
 * Tile autotuning.  The leaves are factored and solved in two size classes
 * (orders up to 192 in FP32, 256 in FP64, and the rest), the small class on
 * the factorization's second stream beside the large one.  The two largest
 * launches of a factorization, the LU of the leaf blocks (Algorithm 1's leaf
 * factorization; the large class, or the small one without large leaves)
 * and the leaf solves of every level's panel columns (Algorithm 2 at the
 * leaves; each class on its own), each have two tile shapes: for the LU a panel width of 16 or 32 and 4 or 8 waves per
 * matrix (8 halves each thread's panel rows and doubles the waves sharing a
 * matrix's trailing update), for the solves 16 or 32 right-hand sides per
 * workgroup (32 reuses each factor tile for twice the columns but needs
 * twice the LDS, so fewer workgroups share a compute unit).  Which is faster
 * depends on the leaf sizes, the ranks and the precision.
 *
 *  INVASKIT_TUNE_AUTO  a launch whose shape class (operation, precision,
 *                      largest order, number of systems and total work, in
 *                      half-octave bins) is not yet in the process-wide
 *                      tuning table is timed with each candidate, twice, on
 *                      the factorization's own data (inputs re-evaluated
 *                      before every trial: both launches work in place);
 *                      the faster is recorded and used from then on by every
 *                      handle.  The first factorization of a new shape class
 *                      therefore takes longer (up to eight extra leaf LUs
 *                      and four extra leaf solves).
 *  INVASKIT_TUNE_OFF   the built-in defaults (LU panel 32 in FP32 and 16 in
 *                      FP64, 4 waves; 16 right-hand sides), no timing.
 * A nonzero leaf_lu_panel, leaf_lu_waves or leaf_trsm_cols fixes that choice
 * whatever `tune` says (the LU's candidates are the pairs that agree with
 * the fixed ones).  Leaf LUs of FP32 orders up to 192 always take the
 * one-wave kernel, for which the LU choices do not apply.  FP64 has no LU
 * with panel 32 at 8 waves (it would spill registers): asking for both is
 * INVASKIT_E_ARG, and the tuner leaves that pair out.  32 right-hand sides need (32 + 1) * elem + 4 bytes of LDS
 * per row of the largest leaf; if that exceeds 160 KiB (FP64 leaves above
 * 611 points) AUTO keeps 16 and a fixed 32 fails with INVASKIT_E_ARG.
 *
 * The level wavefront of Algorithm 1 (the reduced systems of eq. (11) and
 * the sweep that applies them) is tuned per level the same way.  The LU of
 * a level's reduced systems of order up to 192 has two forms: one wave per
 * system (no workgroup barriers, the shorter per-column chain; the FP32
 * default) or four waves per system (the block kernel; the FP64 default),
 * and which wins depends on how many systems the level has; the solves of
 * the sweep take 16 or 32 right-hand sides per workgroup.  Trials rebuild
 * the level's reduced systems before each LU and leave the sweep's inputs
 * untouched, so they run inside the first factorization of a shape class;
 * keys "zgetrf.*" (value 1 one wave, 2 block) and "getrs.*.k1.*".  A
 * nonzero zlu_form or zsolve_cols fixes that choice on every level.
 */
#define INVASKIT_TUNE_AUTO 0
#define INVASKIT_TUNE_OFF  1

typedef struct invaskit_solve_info {
  int32_t iterations;            /* refinement steps x += M^-1 r, the first
                                    (direct) solve included                      */
  int32_t converged;             /* 1 when every column met refine_tol, as
                                    measured by the FP64 product                 */
  double final_rel_residual;     /* max over columns of |b - A x| / |b|, FP64   */
  double unrefined_rel_residual; /* same after the first solve x = M^-1 b       */
  int32_t gmres_iterations;      /* GMRES steps (one M^-1 and one product each) */
  int32_t method;                /* INVASKIT_REFINE_* that produced x: NONE,
                                    IR, or GMRES when GMRES ran                  */
} invaskit_solve_info;

typedef struct invaskit_handle_s* invaskit_handle;

/* Fill *opt with the defaults listed above. */
int invaskit_default_options(invaskit_options* opt);

/*
 * Workspace of a factorization, in bytes: n_lambda = 0 for
 * invaskit_factor, n_lambda >= 1 for invaskit_factor_sweep with that many
 * lambdas (options->lambda_group as it will be passed).  Host only: plans
 * the layout (the factors, W storage, reduced systems, skeleton sweep
 * blocks, descriptor tables) without touching the device.  Same argument
 * checks as invaskit_factor.
 */
int invaskit_factor_workspace_bytes(const invaskit_problem* problem,
                                    const invaskit_options* options, int32_t n_lambda,
                                    size_t* bytes);

/*
 * Factor lambda*I + K~ (Algorithm 1, Factorize, done level by level
 * bottom-up): LU with partial pivoting of every leaf block
 * lambda*I + K_{aa}; for every level k = L..1 the skeleton blocks
 * K_{c, sibling~} (eq. (7)) solved through c's subtree
 * (Algorithm 2) to give W; the reduced systems
 * [[I, P_{r~r} W_{r l~}], [P_{l~l} W_{l r~}, I]] of eq. (11) and
 * their LU.  lambda enters only the leaf diagonal blocks.
 *
 * workspace: DEVICE, ws_bytes >= invaskit_factor_workspace_bytes(problem,
 * options, 0), 256-byte aligned.  The handle keeps its factors and
 * descriptor tables there: the caller must leave it untouched and allocated
 * until invaskit_destroy().  Validates every input on the host before any
 * launch (E_ARG, E_WORKSPACE).  hip_stream may be NULL (the null stream).
 * Part of the work runs on a second stream the handle owns (default
 * priority), ordered after everything already enqueued on hip_stream and
 * joined back into it before the factor's end.  Synchronizes the stream
 * once at the end to read the pivot status: a zero or non-finite pivot
 * returns E_SINGULAR, names the node in invaskit_last_error(), and still
 * returns the handle in *out.
 */
int invaskit_factor(const invaskit_problem* problem, double lambda,
                    const invaskit_options* options, void* workspace, size_t ws_bytes,
                    void* hip_stream, invaskit_handle* out);

/*
 * Factor lambda_i I + K~ for n_lambda values of lambda (Section II-C: only
 * the leaf LU, W and the reduced systems depend on lambda).  The kernel
 * blocks -- the leaf blocks K_aa and the skeleton blocks of every level --
 * are evaluated once, without lambda, into the workspace and shared: each
 * lambda's leaf blocks are copied from them with lambda_i on the diagonal,
 * and its leaf solves read the skeleton blocks from them.  The lambdas are
 * factored in batches of options->lambda_group (0: all at once): every
 * launch of a batch covers all of its lambdas (their leaf LUs in one LU
 * launch, and so on).  out[i] receives the handle for lambdas[i].
 * workspace: ws_bytes >= invaskit_factor_workspace_bytes(problem, options,
 * n_lambda), owned as for invaskit_factor until every handle of the sweep
 * is destroyed.  Arguments, streams and errors as invaskit_factor; every
 * lambda is validated before any work.  Returns the first non-OK status; a
 * handle whose factorization reported E_SINGULAR is still returned, but on
 * any other error no handle is returned (every out[i] is NULL).
 */
int invaskit_factor_sweep(const invaskit_problem* problem, const double* lambdas,
                          int32_t n_lambda, const invaskit_options* options, void* workspace,
                          size_t ws_bytes, void* hip_stream, invaskit_handle* out);

/*
 * Refactor an existing handle for a new lambda (Section II-C, refactoring
 * for a different lambda): skeletons and P are reused, leaf LU, W and the
 * reduced systems are recomputed in the handle's workspace.  A handle of a
 * sweep starts from the sweep's shared kernel blocks (no evaluation).  Same
 * errors as invaskit_factor.
 */
int invaskit_refactor(invaskit_handle handle, double lambda);

/*
 * Scratch of invaskit_solve with nrhs right-hand sides, in bytes: *bytes
 * includes the GMRES bases (gmres_restart + 1 and gmres_restart vectors of
 * n x nrhs FP64), *min_bytes (may be NULL) leaves them out.  invaskit_solve
 * accepts any size from *min_bytes up; GMRES then runs with the longest
 * restart that fits (at least 2), or not at all (refine = GMRES then fails
 * with E_WORKSPACE; AUTO stops where plain refinement stops).  Host only.
 */
int invaskit_solve_workspace_bytes(invaskit_handle handle, int64_t nrhs, size_t* bytes,
                                   size_t* min_bytes);

/*
 * x = (lambda*I + K~)^-1 b (Algorithm 2, Solve, done bottom-up), refined
 * per options->refine (see Refinement modes) until every column satisfies
 * refine_tol.  b, x: DEVICE, FP64, n x nrhs column-major with leading
 * dimensions ldb, ldx >= n; they must not overlap.  E_NOT_CONVERGED if the
 * refinement stops short: x then holds the iterate with the smallest
 * residual (worst column) and info->final_rel_residual that residual.
 * scratch: DEVICE, 256-byte aligned, scratch_bytes as described under
 * invaskit_solve_workspace_bytes, not overlapping b or x.  The first bytes of
 * scratch receive the solve's descriptor tables, which a later call with the
 * same handle, nrhs and scratch pointer reuses without copying them again:
 * between such calls nothing else may write to that scratch (use another
 * buffer for other handles and for invaskit_matvec).  info may be NULL.
 */
int invaskit_solve(invaskit_handle handle, const double* b, int64_t nrhs, int64_t ldb,
                   double* x, int64_t ldx, void* scratch, size_t scratch_bytes,
                   invaskit_solve_info* info);

/* Scratch of invaskit_matvec with nrhs columns, in bytes.  Host only. */
int invaskit_matvec_workspace_bytes(invaskit_handle handle, int64_t nrhs, size_t* bytes);

/*
 * y = (lambda*I + K~) x in FP64, by the ASKIT Skeletonize upward pass and
 * the Evaluate traversal with separation "i not in node" (Section II-B):
 * exact leaf blocks plus K_{i, c~} P_{c~ c} x_c for every node c that
 * does not contain i but whose parent does.  x, y: DEVICE FP64,
 * n x nrhs column-major, must not overlap.  scratch: DEVICE, 256-byte
 * aligned, scratch_bytes >= invaskit_matvec_workspace_bytes; its descriptor
 * tables are reused as for invaskit_solve.
 */
int invaskit_matvec(invaskit_handle handle, const double* x, int64_t nrhs, int64_t ldx,
                    double* y, int64_t ldy, void* scratch, size_t scratch_bytes);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * product of invaskit_matvec with its scratch taken from a static device
 * array of INVASKIT_STATIC_SCRATCH_BYTES inside the library (one per GPU,
 * held until the process ends) instead of a caller buffer.  Allocates
 * nothing.  A product whose scratch (invaskit_matvec_workspace_bytes) exceeds
 * the array fails with INVASKIT_E_WORKSPACE before any launch.  Every call on
 * a GPU, from any handle, shares that GPU's array and rewrites its
 * descriptor tables: calls that overlap on one GPU (other streams, other
 * threads) race.  Arguments and results as invaskit_matvec.
 */
#define INVASKIT_STATIC_SCRATCH_BYTES (64u << 20)
int invaskit_matvec_noalloc(invaskit_handle handle, const double* x, int64_t nrhs, int64_t ldx,
                            double* y, int64_t ldy);

/* Bytes of the workspace the handle's own buffers span (for a handle of a
 * sweep: its region, without the shared kernel blocks). */
int invaskit_device_bytes(invaskit_handle handle, size_t* bytes);

/*
 * Milliseconds spent in the phases of the last factor (HIP events on the
 * stream each phase runs on; [3] runs beside [0] and [1], so the phases need
 * not add up to the total): [0] leaf block evaluation, [1] leaf LU, [2]
 * inverses of the factors' 64 x 64 diagonal blocks (leaves), [3] skeleton
 * blocks, [4] leaf solves, [5] leaf projections, [6] skeleton sweep, [7]
 * host planning of the handle (descriptor tables built and uploaded; wall
 * clock; not part of [9]), [8] reduced systems
 * (assembly, LU, diagonal-block inverses), [9] total, [10] the leaf LU of
 * the large leaves alone (one launch on the caller's stream; [1] adds the
 * small leaves' LU on the second stream), [11] the leaf solves of the large
 * leaves alone (likewise part of [4]).  Writes min(n, 12) values.
 */
int invaskit_phase_times(invaskit_handle handle, double* ms, int32_t n);

/* The tile shapes the last factor of `handle` used (see Tile autotuning). */
typedef struct invaskit_tile_config {
  int32_t leaf_lu_panel;   /* 16 or 32                                          */
  int32_t leaf_lu_waves;   /* 4 or 8                                            */
  int32_t leaf_trsm_cols;  /* 16 or 32: the solves of the large leaves          */
  int32_t tuned;           /* 1 if that factor timed candidates itself          */
  float lu_ms[4];          /* its trial times (best of two) for the LU with
                              (panel, waves) = (16,4), (32,4), (16,8), (32,8)   */
  float trsm_ms[2];        /* and for 16, 32 right-hand sides; 0 if not timed   */
  int32_t leaf_trsm_cols_small; /* 16 or 32: the solves of the small leaves
                              (orders up to 192 in FP32, 256 in FP64); 0 if
                              there are none                                     */
  float trsm_small_ms[2];  /* their trial times for 16, 32; 0 if not timed      */
  int32_t zlu_one_wave_levels; /* bit j set: level j's reduced systems were
                              factored by the one-wave kernel                    */
  int32_t zsolve32_levels; /* bit j set: the sweep at level j took 32
                              right-hand sides per workgroup                     */
  int32_t leaf_pivoting;   /* 1 if the leaf LU used partial pivoting, 0 if the
                              larger leaf blocks were factored without row
                              exchanges                                          */
} invaskit_tile_config;
int invaskit_tile_config_get(invaskit_handle handle, invaskit_tile_config* out);

/*
 * The process-wide tuning table as text, one "key value" line per entry
 * (key: shape class, value: the chosen tile parameter: 16 or 32, for the
 * "getrfw." keys the LU's waves, 4 or 8, for the "zgetrf." keys the reduced
 * systems' LU form, 1 or 2), so that a caller can keep it
 * across processes.  export: writes at most `n` bytes including the
 * terminating NUL into buf (buf may be NULL when n == 0) and sets *needed to
 * the full size including the NUL.  import: adds (or replaces) the entries of
 * `text` in that format; a malformed line, an unknown key prefix or a value
 * out of its key's set fails with INVASKIT_E_ARG and changes nothing.
 * clear: empties the table.
 */
int invaskit_tuning_export(char* buf, size_t n, size_t* needed);
int invaskit_tuning_import(const char* text);
int invaskit_tuning_clear(void);

/* Release the handle (host memory, its second stream and events).  The
 * caller's workspace and borrowed buffers are untouched. */
int invaskit_destroy(invaskit_handle handle);

/* Static text for a status code. */
const char* invaskit_status_string(int status);

/* Copy the last error message of `handle` (or of the calling thread's last
 * handle-less call when handle is NULL) into buf (NUL-terminated). */
int invaskit_last_error(invaskit_handle handle, char* buf, size_t n);

/* ---------------------------------------------------------------------------
 * Batched building blocks, exposed for unit testing and for callers that
 * assemble their own hierarchy.  Each takes a DEVICE workspace for its
 * descriptor tables (and, for the solves, the diagonal-block inverses):
 * called with workspace == NULL it only stores the bytes it needs in
 * *ws_needed and launches nothing; otherwise ws_bytes must be at least that
 * (E_WORKSPACE), and ws_needed may be NULL.  All run on `hip_stream` and
 * synchronize it before returning.
 * ------------------------------------------------------------------------- */

/*
 * LU with partial pivoting (LAPACK getrf semantics: pivot = first row of
 * largest magnitude) of `count` square matrices of uneven order in one
 * launch -- the leaf LU of Algorithm 1 and the LU of the reduced systems.
 *  a        DEVICE, element type dtype; matrix i is n[i] x n[i] row-major
 *           with row stride n[i], starting at element a_offsets[i];
 *           overwritten by the factors of P A = L U with rows left in place:
 *           logical row j of the packed L\U (L unit lower below the
 *           diagonal, U on and above it) is stored in row perm[j].  No row
 *           is moved; invaskit_getrs_batched reads this layout.
 *  a_offsets, n  HOST, count entries; 1 <= n[i] <= 1024.
 *  perm     DEVICE int32, sum(n) entries; matrix i's block starts at the sum
 *           of the preceding n: perm[j] = original row pivoted to position j
 *           (also the storage row of the factors' row j).
 *  info     DEVICE int32, count entries: 0, or j+1 for the first zero or
 *           non-finite pivot in column j.
 */
int invaskit_getrf_batched(int32_t dtype, void* a, const int64_t* a_offsets,
                           const int32_t* n, int32_t count, int32_t* perm,
                           int32_t* info, void* workspace, size_t ws_bytes,
                           size_t* ws_needed, void* hip_stream);

/*
 * Solve A_i X_i = B_i in place with the row-major factors of
 * invaskit_getrf_batched (row permutation, unit-lower L, upper U); the
 * inverses of the factors' 64 x 64 diagonal blocks are formed first, in the
 * workspace.  b: DEVICE, element type dtype; system i has nrhs[i] columns
 * with leading dimension ldb[i] >= n[i] and starts at element b_offsets[i].
 * a_offsets, n, nrhs, ldb, b_offsets: HOST.
 */
int invaskit_getrs_batched(int32_t dtype, const void* a, const int64_t* a_offsets,
                           const int32_t* n, const int32_t* perm, void* b,
                           const int64_t* b_offsets, const int32_t* nrhs,
                           const int64_t* ldb, int32_t count, void* workspace,
                           size_t ws_bytes, size_t* ws_needed, void* hip_stream);

/*
 * Gaussian kernel blocks (eq. (1)): out_i[r, c] =
 * K(x[row0_i + r], x[col_i(c)]) + (diag_i && r == c ? shift : 0), where
 * col_i(c) = cols[cols_offsets[i] + c].  For d <= 64 the squared distances
 * are direct differences in FP64; for d > 64 they come from the Gram form
 * |x'|^2 + |y'|^2 - 2 x'.y' on the FP64 matrix cores, with x' and y'
 * shifted by the tile's first row point (a point against itself gets
 * exactly 0).  points: DEVICE n x d row-major of points_dtype; cols: DEVICE
 * int32; out: DEVICE element type out_dtype, block i is rows_i x ncols_i
 * column-major (ld = rows_i) at element out_offsets[i].  All other arrays
 * HOST, count entries.
 */
int invaskit_kernel_blocks(int32_t points_dtype, const void* points, int32_t d, double h,
                           int32_t out_dtype, void* out, const int64_t* out_offsets,
                           const int64_t* row0, const int32_t* rows,
                           const int32_t* cols, const int64_t* cols_offsets,
                           const int32_t* ncols, const int32_t* diag, double shift,
                           int32_t count, void* workspace, size_t ws_bytes,
                           size_t* ws_needed, void* hip_stream);

/*
 * Grouped GEMM on the matrix cores, C_i = beta*C_i + alpha*A_i B_i for
 * `count` products of different shapes in one launch (the level-synchronous
 * GEMMs of the SMW updates, eq. (11), and of eq. (12)).
 * a, b, c: DEVICE, element type dtype.  Product i: A_i is m[i] x k[i],
 * column-major with leading dimension lda[i] (row-major when a_rowmajor[i]
 * != 0, lda = row stride); B_i is k[i] x n[i] column-major (ldb[i]); C_i is
 * m[i] x n[i] column-major (ldc[i]); element offsets a_off, b_off, c_off.
 * beta == 0 never reads C.  All size arrays HOST, count entries.
 */
int invaskit_gemm_batched(int32_t dtype, const void* a, const void* b, void* c,
                          const int64_t* a_off, const int64_t* b_off, const int64_t* c_off,
                          const int32_t* m, const int32_t* n, const int32_t* k,
                          const int64_t* lda, const int32_t* a_rowmajor, const int64_t* ldb,
                          const int64_t* ldc, double alpha, double beta, int32_t count,
                          void* workspace, size_t ws_bytes, size_t* ws_needed,
                          void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* INVASKIT_H */
