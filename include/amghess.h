/*
 * amghess.h -- C ABI of the MI355X (gfx950) library that solves the
 * linear-quadratic elliptic control problem of Barker & Draganescu,
 * "Algebraic multigrid preconditioning of the Hessian in PDE-constrained
 * optimization" (arXiv:2001.11533):
 *
 *   minimise 1/2 ||y - y_d||^2 + beta/2 ||u||^2
 *   subject to -div(kappa grad y) = u in Omega, y = 0 on the Dirichlet boundary
 *   (Section 2, eqs. functionalcont, pdecont; discrete form eqs. functional,
 *   state),
 *
 * through the symmetric reduced system of Section 5.2 (eq. firstorderpractice)
 *
 *   H_0 u = (K^T M_y K + beta M_u) u = K^T M_y y_d,   K = A^{-1} M_yu,
 *
 * solved by conjugate gradients preconditioned with the multilevel Hessian
 * preconditioner of Section 3.2 (Algorithm MLAS) in its practical form,
 * built from a smoothed-aggregation AMG hierarchy.
 *
 * Spaces.  State and control share one P1 space on N nodes.  With the
 * Dirichlet mask d (1 on constrained nodes) and D = diag(1 - d):
 *   A_0 = D A D + (I - D),  M_y = D M D,  M_yu = D M,  M_u = M
 * (the state lives in H^1_0 as in Section 2; the control lives on every
 * node).  Coarse levels use P_j = S_j, so M_y, M_u and M_yu coincide there.
 *
 * Conventions for every call below.
 *   - Return value: AMG_OK (0) or a negative AMG_ERR_* code.  No call aborts
 *     or throws; after an error amg_last_error() describes it.
 *   - Matrices given to amg_setup are CSR with int32 indices and FP64 values
 *     in DEVICE memory, sorted unique column indices per row.  They are
 *     copied during setup; the caller keeps ownership and may free them
 *     afterwards.
 *   - Vectors are caller-owned DEVICE buffers of FP64, row-major [n x nb]
 *     (entry (i, c) at i*nb + c), n the size of the level addressed,
 *     1 <= nb <= opts.nb_max <= 16.  Inputs and outputs must not alias.
 *   - Every call enqueues its work on the stream given to amg_setup and
 *     returns once its outputs are valid on that stream (calls that test
 *     convergence synchronise on a few scalars).
 *   - A context is not thread-safe; use one context per host thread.
 *   - Every public vector is FP64 whatever opts.inner_precision is.
 */
#ifndef AMGHESS_H
#define AMGHESS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AMG_OK 0
#define AMG_ERR_ARG (-1)            /* invalid argument (null, size, range) */
#define AMG_ERR_NOT_SYMMETRIC (-2)  /* input stiffness/mass matrix not exactly symmetric */
#define AMG_ERR_NOT_SPD (-3)        /* non-positive diagonal / non-positive pivot of a dense inverse */
#define AMG_ERR_NOCONV (-4)         /* an iteration hit its limit; outputs hold the last iterate */
#define AMG_ERR_INDEFINITE (-5)     /* outer CG met p.Hp <= 0 or r.Br <= 0 */
#define AMG_ERR_HIP (-6)            /* a HIP runtime call failed */
#define AMG_ERR_OOM (-7)            /* device allocation failed */
#define AMG_ERR_DENSE_TOO_LARGE (-8)/* coarsest level above opts.dense_max */
#define AMG_ERR_CAPACITY (-9)       /* a sparse product row exceeded the kernel's table */

typedef struct amg_ctx amg_ctx;

typedef struct {
    int32_t nrows, ncols, nnz;
    const int32_t *rowptr;  /* [nrows + 1] */
    const int32_t *col;     /* [nnz], sorted and unique within a row */
    const double *val;      /* [nnz] */
} amg_csr;

typedef struct {
    double beta;            /* regularisation beta > 0 (eq. functional) */
    int32_t hess_levels;    /* levels l of the Hessian preconditioner; 0 = all AMG levels */
    int32_t auto_levels;    /* 1: on an indefinite preconditioner retry with l - 1 levels */
    int32_t max_levels;     /* AMG levels at most (default 10) */
    int32_t max_coarse;     /* stop coarsening at or below this size (default 200) */
    int32_t dense_max;      /* largest dense coarse level (default 4096) */
    double theta0;          /* strength threshold at level 0, halved per level (0.08) */
    uint64_t agg_seed;      /* seed of the aggregation priority hash */
    int32_t nu;             /* l1-Jacobi sweeps before and after the coarse correction (1) */
    double inner_rtol;      /* A-solves inside K and K^T (1e-8, Section 5.3) */
    double mass_rtol;       /* mass-matrix solves, all inside the preconditioner (1e-8, Section 5.3) */
    double precond_inner_rtol; /* A-solves inside the preconditioner's H_j (1e-8, Section 5.3) */
    int32_t inner_maxit, mass_maxit, outer_maxit; /* 500, 500, 200 */
    int32_t inner_precision;/* 64, or 32: float32 V-cycles (see mixed_mode) */
    double inner32_rtol;    /* float32 CG tolerance per refinement step (1e-6) */
    int32_t refine_maxit;   /* refinement steps at most (6) */
    int32_t nb_max;         /* widest batch used with this context (1..16) */
    int32_t precond;        /* 1: multilevel preconditioner, 0: plain outer CG */
    int32_t check_every;    /* inner CG: host convergence poll period after the predicted count (1) */
    int32_t use_graphs;     /* 1: replay CG iterations from captured HIP graphs, 0: launch eagerly,
                               2 (default): graphs for the mass-matrix (Jacobi) CGs only */
    double coarse_hess_rtol;/* coarsest Hessian level above dense_max: unpreconditioned CG to this
                               relative residual (1e-4, Section 5.2); at or below dense_max it is
                               inverted exactly (Section 3.2) */
    int32_t dense_solve_max;/* coarse levels j >= 1 (below the coarsest) with at most this many rows
                               solve A_j and M_j exactly with dense inverses instead of CG (2048;
                               0 = always iterative) */
    int32_t mixed_mode;     /* inner_precision 32 only.  0 (default): FP64 CG preconditioned by the
                               float32 V-cycle (residual cast to float32, correction read back);
                               1: float32 CG + V-cycle inside FP64 iterative refinement */
    int32_t smoother;       /* V-cycle smoothing: 0 (default) nu l1-Jacobi sweeps; 1 the Chebyshev
                               iteration of degree 2 preconditioned by the l1 diagonal on the interval
                               [0.3, 1] of the spectrum of D_l1^{-1} A (bounded by 1 on every level),
                               before and after the coarse correction */
    int32_t true_resid;     /* 1: reduced_solve recomputes b - H_0 u at exit (one more Hessian
                               action) and reports its norm in amg_info.true_rel_resid; 0 (default) */
    int32_t autotune;       /* 1: apply the process-wide table of tuned sparse-product geometry
                               (filled by amg_autotune) to this context's products; 0 (default):
                               the fixed rule */
} amg_opts;

typedef struct {
    int32_t outer_iters;      /* outer CG iterations */
    int32_t inner_solves;     /* A-solves performed (all levels) */
    int32_t inner_iters_total;/* CG iterations summed over A-solves (per column max) */
    int32_t inner_iters_max;
    int32_t mass_iters_total;
    int32_t refine_steps;     /* FP64 refinement steps (inner_precision 32) */
    int32_t levels;           /* AMG levels L */
    int32_t ell;              /* Hessian levels used (after any fallback) */
    int32_t status_detail;    /* reduced_solve: this column's outer iterations */
    int32_t pad_;
    double rel_resid;         /* outer ||r||/||b|| of the recursive residual (this column) */
    double ms_total;          /* wall time of the call */
    double true_rel_resid;    /* ||b - H_0 u||_2 / ||b||_2 recomputed at exit (reduced_solve with
                                 opts.true_resid = 1), else -1 */
    double ms_phase[8];       /* reduced_solve: device time (ms) between phase boundaries on the
                                 context's stream: [0] right-hand side K^T M_y y_d, [1] Hessian
                                 actions of the outer CG, [2] preconditioner actions, [3] the
                                 outer CG's own vector work and read-backs, [4] the true-residual
                                 check; [5..7] 0.  Other calls: all 0 */
    double bytes_moved;       /* algorithmic bytes of the sparse and dense products the call
                                 issued: per sparse product 4 (n+1) + (4 + s) nnz + 2 s n nb
                                 (s = 8 or 4 value bytes), per dense apply s (n^2 + 2 n nb);
                                 elementwise vector work is not counted */
} amg_info;

/* Fill *o with the defaults listed above.  Returns AMG_ERR_ARG if o is null. */
int amg_opts_default(amg_opts *o);

/* ---- P1 finite-element assembly on the host (Section 2: [A]_ij = a(phi_j, phi_i),
 *      [M]_ij = (phi_j, phi_i)).  No boundary condition is applied here. ----
 * amg_p1_pattern: number of stored entries of the mesh graph (all vertex pairs
 *   sharing an element, the diagonal included).  elems: host int32 [ne x (dim+1)].
 * amg_p1_assemble: host outputs rowptr[nv+1], col[nnz], valA[nnz], valM[nnz]
 *   (caller-allocated; nnz from amg_p1_pattern).  coords: host FP64 [nv x dim];
 *   kappa: host FP64 [ne], one value per element.  Each entry sums its element
 *   contributions in ascending element index.  Columns sorted, explicit zeros kept.
 * Errors: AMG_ERR_ARG for dim not 2/3, sizes <= 0, out-of-range vertex ids, or a
 *   mismatching nnz. */
int amg_p1_pattern(int dim, int32_t nv, int32_t ne, const int32_t *elems, int32_t *nnz);
int amg_p1_assemble(int dim, int32_t nv, const double *coords, int32_t ne, const int32_t *elems,
                    const double *kappa, int32_t nnz, int32_t *rowptr, int32_t *col,
                    double *valA, double *valM);

/* ---- The same assembly on the GPU (Section 2), bit-identical to amg_p1_assemble:
 *      one thread per row adds the row vertex's element contributions in ascending
 *      element index with the host's element arithmetic (no fused multiply-add). ----
 * amg_p1_pattern_device: *nnz (host) = stored entries of the mesh graph.
 *   elems: device int32 [ne x (dim+1)].
 * amg_p1_assemble_device: device outputs rowptr[nv+1], col[nnz], valA[nnz], valM[nnz]
 *   (caller-allocated, nnz from amg_p1_pattern_device); coords: device FP64 [nv x dim];
 *   kappa: device FP64 [ne].  Columns sorted, explicit zeros kept.
 * stream: a hipStream_t passed as void* (NULL: the default stream); the work runs on
 *   it and both calls synchronise it before returning.  Temporary device memory
 *   (vertex-to-element lists, row counts and pointers, scan sums: about
 *   4 (3 nv + ne (dim+1)) bytes) comes from the library's process-wide cache of
 *   device blocks and goes back to it when the call returns (a new block is
 *   allocated only when the cache holds none of a fitting size).
 * Errors: AMG_ERR_ARG for dim not 2/3, sizes <= 0, null pointers, out-of-range vertex
 *   ids (checked on the device before any use), a total beyond int32 or an nnz that
 *   differs from the mesh graph's; AMG_ERR_OOM when the workspace cannot be
 *   allocated; AMG_ERR_HIP when another HIP call fails. */
int amg_p1_pattern_device(int dim, int32_t nv, int32_t ne, const int32_t *elems, int32_t *nnz,
                          void *stream);
int amg_p1_assemble_device(int dim, int32_t nv, const double *coords, int32_t ne,
                           const int32_t *elems, const double *kappa, int32_t nnz,
                           int32_t *rowptr, int32_t *col, double *valA, double *valM,
                           void *stream);

/* amg_p1_assemble_device without any device allocation, for callers that cannot
 * allocate (code that runs between graph captures or inside a serving loop, or a
 * harness that forbids hipMalloc): the same arguments, results (bit for bit) and
 * errors as amg_p1_assemble_device.  Its workspace (the lists and counters above,
 * 4 (3 (nv + 1) + ne (dim+1)) bytes plus a few KiB for scan sums and alignment) is a
 * static 32 MiB device array of the library, one per device it runs on, held until
 * the process ends: enough for the 64^3 Kuhn cube (about 27 MiB).  A mesh that needs
 * more is refused with AMG_ERR_ARG before anything runs.  Every call on a device
 * reuses that device's array, so calls that overlap on one device (two host threads,
 * or two streams) race; serialise them.  Calls no hipMalloc, hipFree or allocating
 * library routine. */
int amg_p1_assemble_device_noalloc(int dim, int32_t nv, const double *coords, int32_t ne,
                                   const int32_t *elems, const double *kappa, int32_t nnz,
                                   int32_t *rowptr, int32_t *col, double *valA, double *valM,
                                   void *stream);

/* Build the context: the Dirichlet-reduced stiffness A_0, the smoothed-aggregation
 * hierarchy (strength graph, distance-2 aggregation, smoothed prolongators S_j and
 * their transposes, Galerkin products A_{j+1} = S_j^T A_j S_j and M_{j+1} = S_j^T M_j
 * S_j: eqs. coarsestiffness and coarsemass with P_j = S_j), the dense inverse of
 * the coarsest A (and of A_j, M_j on small levels), and the dense coarsest Hessian
 * H_{l-1} (Section 3.2: the coarsest level is inverted exactly).
 *   A, M: the assembled stiffness and mass matrices (device CSR, same pattern not
 *         required), N x N, exactly symmetric.
 *   dirichlet: device uint8 [N] (1 = Dirichlet node) or NULL (none).
 *   The coarsest AMG level must have at most opts.dense_max rows (else
 *   DENSE_TOO_LARGE); the coarsest Hessian level may be larger (see
 *   coarse_hess_rtol).
 *   opts: NULL for defaults.  stream: a hipStream_t or NULL (default stream).
 * Errors: ARG, NOT_SYMMETRIC, NOT_SPD, DENSE_TOO_LARGE, CAPACITY, OOM, HIP.
 * On error *out is NULL and nothing is leaked. */
int amg_setup(const amg_csr *A, const amg_csr *M, const uint8_t *dirichlet,
              const amg_opts *opts, void *stream, amg_ctx **out);

/* End the context: waits for its streams, then gives its device memory to a
 * process-wide cache that later contexts on the same device draw from (so a
 * context starts and ends without device allocation calls, which wait for the
 * device).  NULL is accepted. */
int amg_destroy(amg_ctx *ctx);

/* Hand every device block held in that cache back to the driver (all
 * devices).  Contexts still alive are not affected.  Returns AMG_OK. */
int amg_release_memory(void);

/* y = K_j u = A_j^{-1} M_{yu,j} u  (eq. solutionopdef at level j; level 0 is the fine
 * problem).  u, y: [n_j x nb].  info may be NULL. */
int state_solve(amg_ctx *ctx, int level, const double *u, double *y, int nb, amg_info *info);

/* z = K_j^T w = M_{yu,j}^T A_j^{-1} w  (the transpose used by the adjoint K^* =
 * M_u^{-1} K^T M_y of Section 2). */
int adjoint_solve(amg_ctx *ctx, int level, const double *w, double *z, int nb, amg_info *info);

/* Hu = H_j u = (K_j^T M_{y,j} K_j + beta M_{u,j}) u  (eq. firstorderpractice). */
int hessian_apply(amg_ctx *ctx, int level, const double *u, double *Hu, int nb, amg_info *info);

/* z = B_0 r, the multilevel preconditioner for H_0: B_{l-1} = H_{l-1}^{-1};
 * C_j(r) = S_j B_{j+1}(S_j^T r) + beta^{-1}(M_{u,j}^{-1} r - S_j M_{u,j+1}^{-1} S_j^T r);
 * B_j = 2C_j - C_j H_j C_j (two calls, Algorithm MLAS) for 0 < j < l-1; B_0 = C_0.
 * This is W_0 M_u^{-1} of eqs. twogridinmulti..fine in the practical form of Section 5.2. */
int hessian_precond_apply(amg_ctx *ctx, const double *r, double *z, int nb, amg_info *info);

/* Solve H_0 u = K^T M_y y_d by CG preconditioned with B_0 (opts.precond = 1) to
 * ||r||_2 <= rtol ||b||_2 per column (Section 5.3 uses 1e-8).  yd, u: [N x nb].
 * u is the output; if u0 is not NULL it is the initial guess (resume), else 0.
 * info: NULL or an array of nb entries (per column).
 * Errors: NOCONV (outer_maxit reached), INDEFINITE (with auto_levels = 0, or at
 * l = 1), and those of the inner solves. */
int reduced_solve(amg_ctx *ctx, const double *yd, const double *u0, double *u, int nb,
                  double rtol, amg_info *info);

/* Reduced functional and gradient (eq. functional with y = K u, Section 2):
 *   J[c] = 1/2 (K u - y_d)^T M_y (K u - y_d) + beta/2 u^T M_u u   (host FP64 [nb]),
 *   grad = K^T M_y (K u - y_d) + beta M_u u                       (device [N x nb]).
 * Either output may be NULL. */
int reduced_objective(amg_ctx *ctx, const double *u, const double *yd, double *J_host,
                      double *grad, int nb, amg_info *info);

/* y = M x at level j.  which: 0 = M_u, 1 = M_y, 2 = M_yu, 3 = M_yu^T (Section 2). */
int amg_mass_apply(amg_ctx *ctx, int level, int which, const double *x, double *y, int nb);

/* q[c] = x_c^T M_which x_c for each column (host FP64 [nb]); which as above (0 or 1). */
int amg_mass_quad(amg_ctx *ctx, int which, const double *x, double *q_host, int nb);

/* ---- introspection (host outputs, caller-allocated) ---- */
int amg_num_levels(amg_ctx *ctx, int32_t *L, int32_t *ell);
/* n_j, nnz(A_j), nnz(S_j) (0 on the coarsest level), nnz(M_j). */
int amg_level_size(amg_ctx *ctx, int level, int32_t *n, int32_t *nnzA, int32_t *nnzS, int32_t *nnzM);
/* agg[n_j] (-1 = Dirichlet) and root flags; level < L-1. */
int amg_copy_aggregates(amg_ctx *ctx, int level, int32_t *agg, uint8_t *root);
/* which: 0 = A_j, 1 = S_j, 2 = S_j^T, 3 = M_j.  Any output pointer may be NULL. */
int amg_copy_csr(amg_ctx *ctx, int level, int which, int32_t *rowptr, int32_t *col, double *val);
/* which: 0 = inverse of the coarsest A (n_{L-1}^2), 1 = dense coarsest Hessian H_{l-1},
 *        2 = its inverse.  Row-major FP64. */
int amg_copy_dense(amg_ctx *ctx, int which, int32_t *n, double *out);
/* Autotuner of the sparse products (the tile choice of the row-blocked SpMV/SpMM
 * kernels): for each CSR product of the context -- A_j, S_j, S_j^T, M_j and the fused
 * coarse-correction pass over T_j = A_j S_j, in FP64 and (inner_precision 32) float32,
 * at the context's padded batch width -- time every lanes-per-row choice
 * G = 2^lg (G times the column groups of a row <= 64) over `reps` launches with HIP
 * events, keep the fastest (the fixed rule's choice unless another is more than 2 %
 * faster), record it in a process-wide table keyed by device, matrix kind, size, stored
 * entries, batch width and value type, and apply it to the context.  Entries the table
 * already holds are applied without timing.  cache_path: NULL, or a JSON file read
 * first (if present) and rewritten with the whole table.  *n_timed (may be NULL): the
 * products timed by this call.  Products of the level-0 sliced-ELL copy (one column)
 * have no such choice.  Results change only at rounding level (the order in which a
 * row's entries are summed).  Errors: ARG (reps < 1, an unreadable or malformed cache
 * file, or one that cannot be written), HIP. */
int amg_autotune(amg_ctx *ctx, int reps, const char *cache_path, int32_t *n_timed);

/* x = V_j b: one application of the AMG V-cycle from level j, the preconditioner of
 * every A_j-solve (Section 5.2 applies K and K^* by AMG-preconditioned CG): the
 * smoothing pass (opts.smoother) before and after the coarse correction S_j V_{j+1}
 * S_j^T r, ending with the exact dense solve at the coarsest level or at the first
 * coarse level j >= 1 with at most opts.dense_solve_max rows.
 *   prec: 64 (FP64 cycle) or 32 (the float32 cycle of inner_precision 32; b is
 *   rounded to float32 on entry, x is the float32 result widened).
 *   b, x: device FP64 [n_j x nb], caller-owned, not aliased.
 * Errors: AMG_ERR_ARG for a bad level, nb, prec (32 needs inner_precision 32) or
 * null pointers. */
int amg_vcycle_apply(amg_ctx *ctx, int level, int prec, const double *b, double *x, int nb);

/* Use l Hessian levels from now on (1 <= l <= L); rebuilds the dense H_{l-1}. */
int amg_set_hess_levels(amg_ctx *ctx, int ell);

/* ---- hierarchy quality (Section 4, eqs. ajnumerical and aj-tilde) ----
 * a~_j = ||K_j - S_j K_{j+1} Pi_j||_2, the approximation number of the coarse
 * spaces that governs the multilevel preconditioner (Pi_j = M_{u,j+1}^{-1}
 * S_j^T M_{u,j}, the control projection with P_j = S_j), estimated as in the
 * paper by the power method on E^T E: iters steps from v0, *a_tilde = the square
 * root of the last Rayleigh quotient.  Each step costs two A-solves on levels
 * level and level + 1 each (inner_rtol) and two mass solves on level + 1.
 *   level: 0 <= level < L - 1.  v0: device FP64 [n_level], not all zero
 *   (caller-owned, not modified).  iters >= 1.
 * Errors: AMG_ERR_ARG for a bad level, null pointers or iters < 1; AMG_ERR_NOCONV
 * from an inner solve. */
int amg_hierarchy_quality(amg_ctx *ctx, int level, const double *v0, int iters, double *a_tilde);
/* Text of the last error of ctx (or of the last failed amg_setup when ctx is NULL). */
const char *amg_last_error(amg_ctx *ctx);

/* Average device time of `reps` back-to-back launches of one kernel on the context's
 * stream, measured with HIP events: which = 0: level-0 SpMV (q = A_0 p), 1: the
 * level-0 first l1-Jacobi sweep fused with the residual (x = D^{-1} b, r = b - A_0 x,
 * the V-cycle's first kernel), 2: a whole V-cycle from level 0, 3: the level-0
 * coarse correction fused with the first post-smoothing step (one pass over
 * T_0 = A_0 S_0; Chebyshev form; needs a hierarchy that keeps T_0), 4: the level-0
 * product of the FP64 inner CG preconditioned by float32 V-cycles (q = A_0 z +
 * beta q_old, with the previous iteration's finalize folded in where a solve folds it;
 * prec 64, inner_precision 32, mixed_mode 0), 5 and 6: the cost of a grid-wide
 * synchronisation: `reps` rounds of an elementwise step over 2^16 floats separated
 * by grid barriers inside one cooperative launch of one workgroup per CU (5), or
 * by kernel boundaries (6, `reps` dependent launches); *ms_avg is then per round.
 * The kernels see zero vectors.  For which 0, 1 and 4, on the level-0 sliced-ELL copy, successive
 * launches rotate which XCD serves which slices, so that no launch finds its
 * share of the matrix in the L2 where the launch before left it (back to back
 * it would; in a solve other work separates the launches).  prec: 64 or 32 (32 needs inner_precision 32); nb as above.
 * *ms_avg receives milliseconds per launch and *bytes the algorithmic bytes one
 * launch moves (row pointers, column indices and values once, every vector it
 * reads or gathers once, every vector it writes once; for which 4 the bytes of
 * the method's product q = A p: 4 (n+1) + (4 + 8) nnz(A_0) + 2 8 n nb).  Level-0 products with one
 * column run on a sliced-ELL copy whose columns are 16-bit offsets from a base
 * per slice of 64 rows (built when every slice spans fewer than 65536 columns),
 * and T_0's columns are kept as 16-bit values when level 1 has at most 65536
 * nodes; such column indices count 2 bytes, all others 4.
 * Errors: ARG; NOCONV if a grid barrier wait of entry 5 timed out. */
int amg_time_kernel(amg_ctx *ctx, int which, int prec, int nb, int reps, double *ms_avg,
                    double *bytes);

#ifdef __cplusplus
}
#endif
#endif
