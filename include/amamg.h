/*
 * amamg.h -- C ABI of the MI355X (gfx950) AM-AMG-preconditioned FGMRES solver for the
 * two-flavour Schwinger-model Wilson-Dirac system D x = psi.
 *
 * Method (arXiv 2608.03515):
 *   - D: Schwinger Model subsection, Wilson operator with U(1) links, two spin components,
 *     sigma_0 = [[0,1],[1,0]], sigma_1 = [[0,-i],[i,0]]; periodic in space, antiperiodic in
 *     time for the fermion field.
 *   - Multigrid setup (Multilevel approach section): coarsening into structured wirebaskets
 *     of aggregate size a and overlap o (SM-AMG subsection, wirebasket figure), interpolation
 *     by the per-wirebasket Schur-complement formula (interpolation equation) with a
 *     normalisation, restriction P^H, Galerkin coarse operator P^H A P.
 *   - Solve: FGMRES right-preconditioned by a V-cycle of the two-level scheme algorithm with
 *     0 pre- and 2 post-smoothing sweeps of a block smoother (Numerical Results section),
 *     relative tolerance 1e-10; the coarsest level is solved directly, or, as in the paper's
 *     experiments (Numerical Results), by unpreconditioned GMRES to a relative tolerance.
 *
 * Conventions
 *   Layout at the boundary (host and device pointers alike):
 *     links  double [2 mu][nt][nx][2 (re,im)]     mu = 0 is the time direction
 *     fields double [nrhs][nt][nx][2 spin][2 (re,im)]
 *     site index t * nx + x; a field is also a complex128 tensor [nrhs][nt][nx][2].
 *   Ownership: the caller owns every buffer it passes; the library copies links at load and
 *     results out at solve.  Handles belong to the library until their *_destroy call.  A
 *     hierarchy keeps its gauge alive: amamg_gauge_destroy fails while hierarchies exist.
 *   Threading: one context = one HIP stream = one host thread at a time; distinct contexts
 *     are independent.  Every call that takes a handle runs on that handle's context stream.
 *   Errors: a negative status means no output was written; amamg_last_error gives a message.
 *     AMAMG_NOT_CONVERGED (> 0) still writes x (the last iterate), info and the history.
 *     Arguments are validated before any device work.
 */
#ifndef AMAMG_H
#define AMAMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMAMG_OK = 0,
  AMAMG_NOT_CONVERGED = 1,            /* iteration cap reached; outputs valid              */
  AMAMG_PENDING = 2,                  /* server: requests still outstanding at the timeout */
  AMAMG_ERR_INVALID_ARG = -1,         /* null pointer, bad enum, handle misuse            */
  AMAMG_ERR_UNSUPPORTED_SHAPE = -2,   /* odd lattice, a does not divide L, o >= a, ...      */
  AMAMG_ERR_OUT_OF_MEMORY = -3,
  AMAMG_ERR_DEVICE = -4,              /* a HIP runtime call failed                          */
  AMAMG_ERR_SINGULAR_LOCAL = -5,      /* zero pivot in a wirebasket or diagonal-block solve */
  AMAMG_ERR_SINGULAR_COARSEST = -6,   /* zero pivot in the coarsest factorisation          */
  AMAMG_ERR_NONFINITE = -7            /* NaN/Inf in links, mass, right-hand side or result  */
} amamg_status;

typedef enum {
  AMAMG_FP64 = 0,                     /* every step in binary64                             */
  AMAMG_MIXED_FP32 = 1,               /* FP32 Arnoldi matvec and V-cycle, FP64 outer loop    */
  AMAMG_MIXED_FP32_BF16LINKS = 2      /* as MIXED_FP32, fine-level smoother links in BF16    */
} amamg_precision;

typedef enum {
  AMAMG_NORM_TESTVEC = 0,             /* least-squares row scale from smoothed test vectors  */
  AMAMG_NORM_CONST = 1,               /* row sums of P equal 1 (constant -> constant)        */
  AMAMG_NORM_NONE = 2
} amamg_norm;

typedef struct {
  int32_t levels;              /* >= 2; the last level is the coarsest (default 2)          */
  int32_t agg_size;            /* a: wirebasket spacing (default 4)                          */
  int32_t overlap;             /* o: shared border width, 1 <= o < a (default 1)             */
  int32_t n_test_vectors;      /* N_v for AMAMG_NORM_TESTVEC, 1..16 (default 4)              */
  int32_t test_vector_sweeps;  /* smoother sweeps on A w = 0 per level (default 4)           */
  int32_t pre_sweeps;          /* default 0                                                  */
  int32_t post_sweeps;         /* default 2                                                  */
  int32_t norm;                /* amamg_norm (default AMAMG_NORM_TESTVEC)                    */
  uint64_t seed;               /* test-vector hash seed (default 0)                          */
  double coarsest_tol;         /* 0: the coarsest level is solved exactly (LU inverse,       */
                               /* default); > 0: unpreconditioned GMRES from 0 to this        */
                               /* relative tolerance, FP64, as in the paper's experiments     */
                               /* (Numerical Results: 0.1); needs <= 2048 coarsest unknowns   */
  int32_t coarsest_max_iters;  /* GMRES steps at most, 1..32 (default 32)                    */
  int32_t block_smoother;      /* FP32 sweeps of levels with 8 x 8 blocks: 0 matrix cores     */
                               /* from 32 x 32 nodes, vector kernels below (default); 1 matrix */
                               /* cores; 2 vector kernels.  Fixed per hierarchy, so results do */
                               /* not depend on the batch                                      */
  int32_t aug_vectors;         /* k >= 0 (default 0): the finest level's coarse space is        */
                               /* augmented with the first k test vectors (Conclusion: test   */
                               /* vectors in the SM-AMG method to capture the near-kernel):   */
                               /* every wirebasket gets k coarse dofs on its node, after its  */
                               /* o^2 b vertex dofs, spanned by an orthonormal basis (Gram-    */
                               /* Schmidt in test-vector order) of the parts of those vectors */
                               /* the wirebasket interpolation leaves on the non-vertex rows  */
                               /* it owns.  Needs AMAMG_NORM_TESTVEC and k <= n_test_vectors; */
                               /* level 1 then has o^2 * 2 + k dofs per node, a power of two  */
                               /* <= 64 unless it is the coarsest level                       */
  int32_t reserved;            /* 0                                                           */
} amamg_setup_params;

typedef struct {
  int32_t restart;             /* FGMRES restart length m, 1..31 (default 20)                */
  int32_t max_iters;           /* cap on Arnoldi steps per right-hand side (default 10000)   */
  double rel_tol;              /* ||psi - D x|| <= rel_tol ||psi|| (default 1e-10)           */
  int32_t precision;           /* amamg_precision (default AMAMG_FP64)                       */
  int32_t use_initial_guess;   /* nonzero: x holds x0 on entry (default 0)                   */
  int32_t groups;              /* the right-hand sides are split into this many batches that  */
                               /* run concurrently on separate HIP streams, overlapping one   */
                               /* batch's latency-bound coarse levels with another's          */
                               /* bandwidth-bound work; 0 or 1 = one batch on the context     */
                               /* stream (default 1, at most 16)                              */
  int32_t graphs;              /* nonzero: each batch captures its restart cycle (the same   */
                               /* kernels every cycle) into a HIP graph and replays it, also  */
                               /* in later calls while the hierarchy's setup, the buffers,   */
                               /* the stream and these parameters are unchanged; bitwise the */
                               /* same results.  Ignored on the null stream, while the kernel */
                               /* timer runs and with pre-smoothing (default 0)               */
} amamg_solve_params;

typedef struct {
  int32_t iterations;          /* Arnoldi steps                                              */
  int32_t restarts;            /* completed cycles that did not converge                     */
  int32_t converged;           /* 1 if the true relative residual met rel_tol                */
  int32_t reserved;            /* padding, written as 0                                      */
  double true_rel_residual;    /* ||psi - D x|| / ||psi|| in FP64 at the end                 */
} amamg_solve_info;

typedef struct amamg_context amamg_context;
typedef struct amamg_gauge amamg_gauge;
typedef struct amamg_hierarchy amamg_hierarchy;

/* Fill defaults (values listed above). */
void amamg_default_setup_params(amamg_setup_params *p);
void amamg_default_solve_params(amamg_solve_params *p);

/* Context on HIP device `device`.  hip_stream: a hipStream_t to run on (borrowed, not
 * destroyed), or NULL for a stream the library creates and owns. */
amamg_status amamg_context_create(int device, void *hip_stream, amamg_context **out);
amamg_status amamg_context_destroy(amamg_context *ctx);
/* Message for the last failure on this context (static storage owned by the context). */
const char *amamg_last_error(const amamg_context *ctx);

/* Load gauge links (host pointer, layout above, |U| = 1 expected but not required) and the
 * bare mass m0 of D (Schwinger Model subsection).  nt, nx even and >= 4. */
amamg_status amamg_gauge_load(amamg_context *ctx, int32_t nt, int32_t nx, const double *links,
                              double m0, amamg_gauge **out);
/* Change m0; hierarchies built from this gauge keep the mass they were built with. */
amamg_status amamg_gauge_set_mass(amamg_gauge *g, double m0);
/* Replace the links (host pointer, same layout and size as at load).  Hierarchies keep their
 * operators until amamg_hierarchy_update. */
amamg_status amamg_gauge_update_links(amamg_gauge *g, const double *links);
amamg_status amamg_gauge_destroy(amamg_gauge *g);

/* AM-AMG setup (Multilevel approach section: coarsening, interpolation, Galerkin operator)
 * with aggregate size and overlap from params (NULL: defaults).  Runs on the GPU. */
amamg_status amamg_setup(amamg_gauge *g, const amamg_setup_params *params, amamg_hierarchy **out);
/* Re-run the setup of an existing hierarchy in place, from the gauge's current links and mass
 * and the parameters it was created with.  Reuses the hierarchy's device memory: after the
 * first setup it allocates nothing.  Same errors as amamg_setup; on error the hierarchy must
 * not be used for solves until an update succeeds. */
amamg_status amamg_hierarchy_update(amamg_hierarchy *h);
/* Move a built hierarchy to bare mass m0 without a new setup.  The wirebaskets, test vectors
 * and interpolation P_k built at the old mass are kept; the operators become those of the new
 * mass: D(m0) on the fine level (Schwinger Model subsection: m0 enters D only on the diagonal)
 * and A_{k+1} = P_k^H A_k P_k above (Multilevel approach: Galerkin operator), computed exactly
 * as A_{k+1} + (m0 - m0_old) G_{k+1} with G_1 = P_0^H P_0 and G_{k+1} = P_k^H G_k P_k (built on
 * the first call and kept with the hierarchy).  The smoother blocks, the coarsest inverse and
 * the FP32 copies are recomputed; solves afterwards use m0.  The gauge's own mass is not
 * changed.  Synchronous on the context stream; must not overlap a solve on this hierarchy.
 * Errors: AMAMG_ERR_INVALID_ARG for a non-finite m0 (nothing changed); AMAMG_ERR_SINGULAR_LOCAL
 * / AMAMG_ERR_SINGULAR_COARSEST when a diagonal block or the coarsest matrix is singular at
 * m0: the hierarchy then holds the new operators and must be moved again (or updated) before
 * the next solve. */
amamg_status amamg_hierarchy_set_mass(amamg_hierarchy *h, double m0);
/* A new hierarchy at bare mass m0 derived from `base` (same passages as set_mass): it shares
 * base's wirebaskets, test vectors, interpolation and mass terms (read only; no copy) and owns
 * its operators, smoother blocks, coarsest inverse and FP32 copies, so several masses of one
 * gauge field can be solved at once for about the memory of their coarse operators.  Equal to
 * a copy of base moved by amamg_hierarchy_set_mass(m0).  base must be a hierarchy made by
 * amamg_setup; while derived hierarchies exist it cannot be destroyed, updated or moved
 * (AMAMG_ERR_INVALID_ARG).  A derived hierarchy can be moved with set_mass, solved and
 * destroyed, but not updated.  Synchronous on the context stream.  Errors as set_mass (on
 * error nothing is created). */
amamg_status amamg_hierarchy_derive_mass(amamg_hierarchy *base, double m0, amamg_hierarchy **out);
/* INVALID_ARG while hierarchies derived from h exist. */
amamg_status amamg_hierarchy_destroy(amamg_hierarchy *h);

/* Solve D x = psi (Schwinger Model subsection: the Wilson-Dirac system) for nrhs right-hand
 * sides with FGMRES right-preconditioned by the AM-AMG V-cycle (Multilevel approach: two-level
 * scheme algorithm, applied recursively; Numerical Results: FGMRES to the relative tolerance,
 * 2 post-smoothing steps).  psi, x: host pointers, layout above; x holds x0 on entry when
 * params->use_initial_guess is set, else it is only written.  info: array of nrhs entries
 * (may be NULL).  Returns AMAMG_NOT_CONVERGED if any right-hand side hit the iteration cap
 * (x, info and the history are still written), AMAMG_ERR_NONFINITE for a non-finite psi
 * (nothing written).  Blocks until the solve has finished. */
amamg_status amamg_solve(amamg_hierarchy *h, int32_t nrhs, const double *psi, double *x,
                         const amamg_solve_params *params, amamg_solve_info *info);
/* Same solve on device pointers (resident in HBM, same layout, 16-byte aligned, else
 * AMAMG_ERR_INVALID_ARG; they stay the caller's).  hip_stream: a hipStream_t whose queued work
 * the solve must follow (it reads psi and x0 after that work), or NULL; the kernels run on
 * the context stream (and, with groups > 1, on streams the hierarchy creates, ordered after
 * the context stream).  Returns after the solve has finished, so work the caller queues on
 * hip_stream afterwards sees x. */
amamg_status amamg_solve_device(amamg_hierarchy *h, int32_t nrhs, const void *psi_dev,
                                void *x_dev, const amamg_solve_params *params,
                                amamg_solve_info *info, void *hip_stream);

/* Residual history of right-hand side `rhs` of the last solve (FGMRES, Numerical Results:
 * relative residual of the outer solver): one entry per Arnoldi step (the FGMRES estimate
 * |g_{j+1}| / ||psi||) and one per cycle end (the true relative residual ||psi - D x|| /
 * ||psi||, flagged 1 in is_true_residual).  Writes min(capacity, length) entries of out and
 * of is_true_residual (either may be NULL); n_written (may be NULL) receives the full length.
 * AMAMG_ERR_INVALID_ARG for an rhs outside the last solve. */
/* Several lattices solved together (spec: uneven lattices batched in one launch): nlat
 * hierarchies, distinct and of one context, each with nrhs[l] right-hand sides in its own
 * device buffers psi_dev[l], x_dev[l] (layout and alignment as amamg_solve_device).  The
 * lattices advance in lock step: at every Arnoldi step each lattice's V-cycle and matvec run on
 * one of up to four streams, then each Gram-Schmidt kernel runs once for all lattices (the
 * Multilevel approach's V-cycle and the FGMRES of Numerical Results, as amamg_solve).  With
 * params->graphs a whole restart round of all lattices is one captured HIP graph, launched once
 * per round.  A right-hand side's result is bitwise that of amamg_solve_device on its lattice
 * alone with nrhs[l] right-hand sides.  info: sum of nrhs entries in lattice order (may be
 * NULL); residual histories per hierarchy as after amamg_solve.  Runs after the work queued on
 * hip_stream (NULL: the context stream), which then follows the solve; blocks until done.
 * Errors as amamg_solve_device; INVALID_ARG for a hierarchy listed twice or of another
 * context. */
amamg_status amamg_solve_multi_device(amamg_hierarchy *const *hs, int32_t nlat, const int32_t *nrhs,
                                      const void *const *psi_dev, void *const *x_dev,
                                      const amamg_solve_params *params, amamg_solve_info *info,
                                      void *hip_stream);
amamg_status amamg_residual_history(const amamg_hierarchy *h, int32_t rhs, double *out,
                                    int32_t capacity, int32_t *n_written,
                                    int32_t *is_true_residual);

/* ---- measurement ------------------------------------------------------------------------- */
typedef enum {
  AMAMG_KT_OFF = 0,
  AMAMG_KT_FINE_MATVEC = 1,   /* Arnoldi D z on the fine lattice                            */
  AMAMG_KT_FINE_GS = 2,       /* one colour of the fine red-black Gauss-Seidel sweep        */
  AMAMG_KT_RESTRICT0 = 3,     /* fine-level restriction, per-wirebasket pass                 */
  AMAMG_KT_PROLONG0 = 4,      /* fine-level prolongation                                     */
  AMAMG_KT_COARSE_GS = 5,     /* one colour of the level-1 block Gauss-Seidel sweep          */
  AMAMG_KT_DOTS = 6,          /* every Gram-Schmidt projection pass V^H w (k_dots)            */
  AMAMG_KT_UPDATE = 7         /* every w -= V h pass (k_update, with its fused projection or  */
                              /* norm)                                                         */
} amamg_kernel_family;
/* Benchmark hook: from now on, bracket every solve-phase launch of the families whose bits
 * (1 << family) are set in family_mask (0 stops) with HIP events on the context stream, and
 * count algorithmic bytes: the bytes the operation must move once -- its fields per
 * right-hand side it served, plus once per launch the operators all of them share (links,
 * interpolation weights, coarse blocks).  Resets all totals. */
amamg_status amamg_kernel_timer(amamg_context *ctx, uint32_t family_mask);
/* Totals of one family since the last amamg_kernel_timer call: launches that served at least
 * one right-hand side, their summed event time in ms and their summed algorithmic bytes. */
amamg_status amamg_kernel_timer_read(const amamg_context *ctx, int32_t family, int64_t *launches,
                                     double *total_ms, double *algorithmic_bytes);

/* ---- launch-shape autotuning ----------------------------------------------------------
 * Some kernels take a launch shape that does not change their arithmetic: the fine smoother's
 * tile width (16, 32 or 64 sites) and, for the FP32 block smoother on levels with 8 x 8 blocks
 * (matrix cores), the stencil offsets per load batch (8, 12 or 24).  Results are bitwise the
 * same for every choice.  AMAMG_TUNE_AUTO (default): the first solve with a new (grid, block size, precision,
 * batch size) times the candidates on its workspace vectors before any right-hand side is
 * admitted and keeps the fastest in the context; AMAMG_TUNE_OFF: fixed defaults;
 * AMAMG_TUNE_FORCE: candidate number `force` of each tunable (clamped), for tests. */
typedef enum { AMAMG_TUNE_AUTO = 0, AMAMG_TUNE_OFF = 1, AMAMG_TUNE_FORCE = 2 } amamg_tune_mode;
typedef struct {
  int32_t kind;          /* 0 fine smoother tile width, 1 block-smoother launch shape          */
  int32_t lt, lx, b;     /* grid and dofs per node of the level                                */
  int32_t precision;     /* amamg_precision of the solve                                      */
  int32_t nrhs;          /* batch size (right-hand-side slots)                                */
  int32_t choice;        /* chosen candidate value                                            */
  int32_t ncand;         /* candidates timed (at most 8)                                      */
  int32_t cand[8];
  double us[8];          /* their measured times in microseconds                              */
} amamg_tune_entry;
amamg_status amamg_context_set_tuning(amamg_context *ctx, int32_t mode, int32_t force);
/* Copies up to `cap` of the context's tuned entries to out (may be NULL with cap 0) and
 * returns their total number in *count. */
amamg_status amamg_tuning_entries(amamg_context *ctx, amamg_tune_entry *out, int32_t cap,
                                  int32_t *count);

/* ---- test hooks (host buffers) ---------------------------------------------------------- */
/* out = D in for nrhs fields at the given precision (FP64 or FP32 links): the Wilson-Dirac
 * operator of the Schwinger Model subsection with its boundary conditions (periodic links,
 * antiperiodic fermions in time).  Layout above; INVALID_ARG for null pointers or nrhs < 1. */
amamg_status amamg_apply_dirac(amamg_gauge *g, int32_t precision, int32_t nrhs,
                               const double *in, double *out);
/* out = D in on device buffers (same layout) at the given precision: AMAMG_FP64 uses FP64
 * fields and links; the mixed modes use FP32 fields ([nrhs][nt][nx][2][2] float) with FP32
 * or BF16 links.  Both pointers must be 16-byte aligned (else AMAMG_ERR_INVALID_ARG).
 * Asynchronous on the context stream. */
amamg_status amamg_apply_dirac_device(amamg_gauge *g, int32_t precision, int32_t nrhs,
                                      const void *in_dev, void *out_dev);
/* The setup's batched dense solve (SM-AMG subsection: the local block systems of the
 * wirebasket interpolation; Multilevel approach: the exact coarsest-level solve): for each of
 * nsys systems the row-major augmented matrix [A | B] of n rows and n + nrhs complex columns
 * (double [nsys][n][n + nrhs][2], host buffer) is overwritten on return with B replaced by
 * A^-1 B (LU with partial pivoting; the other columns then hold factors).  info[sys] = 0, or
 * k + 1 when pivot column k is zero or not finite (that system's B is then not a solution).
 * The same launches as the setup: one workgroup per system for n <= 256 with 32 or more
 * systems (or n <= 64), else panel, interchange and tile launches.  Synchronous; allocates
 * its device buffers.  AMAMG_ERR_INVALID_ARG for n < 1, nrhs < 1, nsys < 1 or null pointers. */
amamg_status amamg_dense_solve(amamg_context *ctx, int32_t n, int32_t nrhs, int32_t nsys, double *aug,
                               int32_t *info);
/* Grid of level `level` (0 = fine lattice) and degrees of freedom per node. */
amamg_status amamg_level_info(const amamg_hierarchy *h, int32_t level, int32_t *lt,
                              int32_t *lx, int32_t *b);
/* Wirebasket classification of level `level` (not the coarsest; SM-AMG subsection and its
 * wirebasket figure: function types by the number of wirebaskets sharing a point, a shared
 * point interpolated from the wirebasket it was assigned to first): per grid point the kind
 * (0 interior, 1 edge, 2 vertex), the primary wirebasket (-1 for vertices) and the coarse
 * node of a vertex (-1 otherwise).  Arrays of lt*lx entries, caller-owned host buffers. */
amamg_status amamg_get_aggregates(const amamg_hierarchy *h, int32_t level, int8_t *kind,
                                  int32_t *owner, int32_t *node);
/* Interpolation rows of level `level`: double [lt*lx][b][4*bc][2]; row (p, i) holds the
 * weights of the 4 corner nodes of p's primary wirebasket W(I,J), corner c = 2*ct + cx is
 * node ((I+ct) mod, (J+cx) mod), column c*bc + j.  Vertex rows are zero (identity). */
amamg_status amamg_get_prolongator(const amamg_hierarchy *h, int32_t level, double *out);
/* Operator of level `level` >= 1: if not coarsest, double [lt*lx][25][b][b][2], block of
 * offset (dt, dx) in [-2,2]^2 at index (dt+2)*5 + (dx+2) couples node n to node n+(dt,dx);
 * at the coarsest level the dense matrix double [n][n][2], n = lt*lx*b. */
amamg_status amamg_get_coarse_operator(const amamg_hierarchy *h, int32_t level, double *out);
/* Transfers between level `level` and the next coarser one (Multilevel approach: restriction
 * P^H, prolongation P) for nrhs vectors on host buffers, with the kernels the V-cycle of the
 * given precision runs (AMAMG_FP64, or AMAMG_MIXED_FP32 with FP32 interpolation weights and
 * FP32 accumulation).  direction 0: out = P^H in, in double [nrhs][n_level][2] (read as FP64, as
 * the fine level's restriction reads the Krylov vector), out double [nrhs][n_coarse][2];
 * direction 1: out = P in, in double [nrhs][n_coarse][2] (rounded to the precision's type),
 * out double [nrhs][n_level][2].  n = lt*lx*b of the level.  Synchronous; allocates its
 * device buffers.  AMAMG_ERR_INVALID_ARG for the coarsest level or a bad direction. */
amamg_status amamg_apply_transfer(amamg_hierarchy *h, int32_t level, int32_t precision,
                                  int32_t direction, int32_t nrhs, const double *in, double *out);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): amamg_apply_transfer on device buffers, allocating
 * nothing.  in_dev, out_dev: caller-owned device buffers, 16-byte aligned, [nrhs][n][2];
 * direction 0 (out = P^H in): in double (FP64, as the V-cycle's fine restriction reads it),
 * out in the precision's type (double for AMAMG_FP64, float for AMAMG_MIXED_FP32);
 * direction 1 (out = P in): in and out in the precision's type.  Asynchronous on the context
 * stream; the same kernels as amamg_apply_transfer, so bitwise its results.  The restriction's
 * partial sums (bytes: complex size x nrhs x wirebaskets x row chunks x 4 o^2 b) go to a fixed
 * library array of AMAMG_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; a call
 * that needs more is refused with AMAMG_ERR_INVALID_ARG before any device work (split the
 * right-hand sides).  Calls that overlap on one GPU (other contexts or streams) share that
 * array and race: order them on one stream. */
#define AMAMG_NOALLOC_SCRATCH_BYTES (64u << 20)
amamg_status amamg_apply_transfer_noalloc(amamg_hierarchy *h, int32_t level, int32_t precision,
                                          int32_t direction, int32_t nrhs, const void *in_dev,
                                          void *out_dev);
/* Post-smoothing sweeps of level `level` (not the coarsest) with the kernels the V-cycle of the
 * given precision runs (Numerical Results: block smoother; point-block multicolour Gauss-Seidel,
 * the fine level red-black, coarse levels 16 colours in the sweep order), in place:
 * x <- sweeps of x_n += A_nn^{-1} (f - A x)_n.  f, x double [nrhs][n_level][2]; x is rounded
 * to the precision's type on entry, f too below the fine level (where the V-cycle's right-hand
 * side is the FP64 Krylov vector).  Default launch shapes (the tuner is not consulted).
 * Synchronous; allocates its device buffers.  sweeps in [1, 16]. */
amamg_status amamg_apply_smoother(amamg_hierarchy *h, int32_t level, int32_t precision, int32_t nrhs,
                                  int32_t sweeps, const double *f, double *x);
/* Smoothed test vectors of level `level`: double [n_test_vectors][lt*lx*b][2]. */
amamg_status amamg_get_test_vectors(const amamg_hierarchy *h, int32_t level, double *out);

/* ---- serving: continuous batching of solve requests ------------------------------------
 *
 * A server owns its device objects (a context on `device`, the gauge fields added to it, the
 * AM-AMG hierarchies it builds, solver instances) and one worker thread that drives them.
 * A request asks for D(m0) x = psi on one of the server's gauge fields, with the given setup
 * parameters (aggregate size, overlap, levels, ...; Multilevel approach and SM-AMG sections),
 * for 1..slots right-hand sides; solve parameters (precision, restart, tolerance, cap) are the
 * server's.  Hierarchies are built on first use per (gauge, m0, setup parameters) by a builder
 * thread on its own stream (running instances keep iterating meanwhile), kept resident and
 * evicted least recently used when the device-memory budget would be exceeded.
 * Each solver instance is a batch of `slots` right-hand-side slots on its own HIP stream,
 * bound to one hierarchy; requests join a running instance at its next restart-cycle
 * boundary as slots free up (continuous batching), and instances bound to different
 * hierarchies run concurrently.  A right-hand side's arithmetic does not depend on the other
 * requests: results are bitwise the same alone and in any mix.
 *
 * Threading: every server call may be made from any thread.  Ownership: psi is copied at
 * submission; x (host, [nrhs][nt][nx][2][2] double) must stay valid until the request is
 * returned by amamg_server_poll.  Errors of one request (non-finite input, failed setup,
 * budget too small for it) are reported in its amamg_request_info.status; a device failure
 * fails every request in flight. */
typedef struct amamg_server amamg_server;

typedef struct {
  int32_t slots;               /* right-hand-side slots per solver instance (default 16, <= 256) */
  int32_t max_instances;       /* solver instances, one HIP stream each (default 4, <= 16)      */
  int32_t precision;           /* amamg_precision of every solve (default AMAMG_MIXED_FP32)     */
  int32_t restart;             /* FGMRES(m) (default 20)                                        */
  int32_t max_iters;           /* Arnoldi steps per right-hand side (default 10000)             */
  int32_t builders;            /* hierarchy builder threads, one stream each (default 2, <= 8)  */
  int32_t graphs;              /* nonzero: instances replay their restart cycle from a HIP      */
                               /* graph captured once per hierarchy binding (default 0)       */
  double rel_tol;              /* default 1e-10                                                 */
  uint64_t hbm_budget;         /* device bytes for hierarchies and instance workspaces;         */
                               /* 0 = three quarters of the free memory at creation           */
} amamg_server_params;

typedef struct {
  uint64_t id;                 /* from amamg_server_submit                                      */
  int32_t status;              /* AMAMG_OK, AMAMG_NOT_CONVERGED or a negative error             */
  int32_t nrhs;
  int32_t iterations;          /* maximum over its right-hand sides                             */
  int32_t converged;           /* 1 if every right-hand side converged                          */
  double true_rel_residual;    /* maximum over its right-hand sides                             */
  double t_submit, t_admit, t_done;   /* server clock, seconds                                  */
  int32_t instance;            /* solver instance that ran it (-1: never admitted)              */
  int32_t hierarchy_built;     /* 1 if its admission built a hierarchy                          */
} amamg_request_info;

typedef struct {
  int64_t setups, evictions;   /* hierarchies built and evicted so far                         */
  uint64_t resident_bytes;     /* hierarchies + instance workspaces now                        */
  uint64_t hierarchy_bytes;    /* of which cached hierarchies                                  */
  uint64_t peak_resident_bytes;
  uint64_t budget_bytes;
  int64_t outstanding;         /* submitted, not yet finished                                   */
  double clock;                /* server clock now, seconds                                     */
  uint64_t last_estimate_bytes;/* bytes reserved for the last hierarchy build (setup and         */
                               /* instance workspace)                                          */
  double setup_seconds;        /* total and longest hierarchy build time                        */
  double setup_seconds_max;
  int64_t derivations;         /* hierarchies derived at another mass (not counted in setups)  */
  double derive_seconds;       /* total and longest derivation time                             */
  double derive_seconds_max;
} amamg_server_counters;

void amamg_server_default_params(amamg_server_params *p);
amamg_status amamg_server_create(int32_t device, const amamg_server_params *params,
                                 amamg_server **out);
/* Finishes every submitted request, then releases everything. */
amamg_status amamg_server_destroy(amamg_server *s);
/* Copy a gauge field (layout above) to the device; gauge_id names it in requests. */
amamg_status amamg_server_add_gauge(amamg_server *s, int32_t nt, int32_t nx, const double *links,
                                    int32_t *gauge_id);
/* Give gauge gauge_id a reference mass: requests submitted on it afterwards are solved with a
 * hierarchy set up once at m_ref and derived from it at each request's mass
 * (amamg_hierarchy_derive_mass: interpolation from m_ref, operators at the request's mass,
 * Multilevel approach section) instead of a setup per mass.  Which hierarchy a request gets
 * depends only on its gauge, mass, setup parameters and this reference mass, so results stay
 * bitwise the same alone and in any mix.  m_ref = NaN restores setups per mass (the default).
 * INVALID_ARG for an unknown gauge or an infinite m_ref. */
amamg_status amamg_server_set_reference_mass(amamg_server *s, int32_t gauge_id, double m_ref);
/* Queue a request; setup NULL = amamg_default_setup_params. */
amamg_status amamg_server_submit(amamg_server *s, int32_t gauge_id, double m0,
                                 const amamg_setup_params *setup, int32_t nrhs, const double *psi,
                                 double *x, uint64_t *request_id);
/* Hand back up to `capacity` finished requests (oldest first); their x is written. */
amamg_status amamg_server_poll(amamg_server *s, amamg_request_info *out, int32_t capacity,
                               int32_t *n_written);
/* Block until no request is outstanding (AMAMG_OK) or timeout_s passed (AMAMG_PENDING). */
amamg_status amamg_server_wait(amamg_server *s, double timeout_s);
amamg_status amamg_server_stats(amamg_server *s, amamg_server_counters *out);
const char *amamg_server_last_error(amamg_server *s);

#ifdef __cplusplus
}
#endif
#endif /* AMAMG_H */
