/*
 * cascade.h - C ABI of the MI355X (gfx950) cascading-smoother multigrid library.
 *
 * The library implements, on one GPU, the method of R. I. Saye, "Cascading
 * Smoothers for Multigrid" (arXiv 2606.12577):
 *   - the setup that fits each cascade level's block-diagonal smoother
 *     Lambda_l by Frobenius-norm minimisation of the error propagator
 *     (Sec. 2.1 additive, Sec. 2.2 multicoloured, Sec. 2.3 elliptic prescaling,
 *     Algorithm 2 and the supplementary multicoloured algorithm);
 *   - the geometric-multigrid V-cycle of Algorithm 1 with forward/reverse
 *     cascade applications (Sec. 2.1 / 2.2 forward formulas, Sec. 2.4 reverse
 *     formulas and the FF / RF solver classes), restriction r_scale * P^T,
 *     correction x <- x - P x_c and a direct solve on the bottom level;
 *   - a stationary solve in FP64 iterative refinement around the V-cycle.
 *
 * Conventions shared by every entry point
 *   - Every function returns cs_status (CS_OK = 0); no C++ exception crosses
 *     the ABI.  On failure cs_last_error(ctx) holds a message and output
 *     buffers are left unspecified unless stated otherwise.
 *   - A context owns every device buffer it allocates and frees them in
 *     cs_destroy.  The caller owns every pointer it passes in; the library
 *     copies host inputs before returning and never frees caller memory.
 *   - Work is issued on the HIP stream given to cs_create (NULL = the null
 *     stream).  Calls on one context must not overlap; distinct contexts
 *     may be used from distinct threads.
 *   - Vectors (right-hand sides, solutions) are device pointers to FP64 arrays
 *     of shape [n][nrhs]: the nrhs values of scalar unknown k are contiguous
 *     at offset k*nrhs.
 *   - Block i of a level owns the contiguous scalar unknowns
 *     [i*block_size, (i+1)*block_size) (the paper's partition A_ij, Sec. 2).
 */
#ifndef CASCADE_H
#define CASCADE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CS_ABI_VERSION 4

typedef struct cs_ctx_s *cs_ctx;

typedef enum {
    CS_OK = 0,
    CS_EINVAL = -1,     /* bad argument, inconsistent sizes, non-positive diagonal */
    CS_ENOMEM = -2,     /* device allocation failed */
    CS_EDEVICE = -3,    /* a HIP runtime call or kernel launch failed */
    CS_ESINGULAR = -4,  /* a normal-equation matrix had no usable pivot */
    CS_ECOLOR = -5,     /* supplied colouring is not proper for the block graph */
    CS_ENOCONV = -6,    /* solve stopped at maxit; x holds the last iterate */
    CS_ESTATE = -7,     /* call out of order (e.g. vcycle before setup) */
    CS_ENAN = -8,       /* NaN or Inf met in the solve */
    CS_EVERSION = -9,   /* saved setup has another format version */
    CS_EIO = -10        /* file could not be read or written */
} cs_status;

typedef enum { CS_ADDITIVE = 0, CS_MULTIPLICATIVE = 1 } cs_mode;   /* Sec. 2.1 / 2.2 */
typedef enum { CS_FF = 0, CS_RF = 1 } cs_order;   /* pre-smoother forward / reverse; post is forward (Sec. 2.4) */
/* V-cycle working precision.  CS_BF16: FP32 vectors and arithmetic, with A and
 * Lambda of 16x16-block levels stored in BF16 and applied on the matrix cores
 * (FP32 accumulation) in the multicoloured sweeps when the solve has one
 * right-hand side; everything else, including the residual restricted to the
 * coarse level (FP32 A), as CS_FP32.  Cascades whose blocks cancel nearly
 * dependent directions need the regularised fit (cs_options.ridge) to converge
 * with BF16 blocks. */
typedef enum { CS_FP64 = 0, CS_FP32 = 1, CS_BF16 = 2 } cs_precision;
/* Where cs_setup takes the smoother of every level from.  CS_SRC_FROBENIUS:
 * the cascade fit of Alg. 2 (the paper's method).  CS_SRC_JACOBI: the
 * reference smoother the cascade is measured against (Sec. 2.1, Sec. 3.2):
 * every cascade level Lambda_l = jacobi_omega * A_ii^{-1}, i.e. nu damped
 * block Jacobi steps (additive) or block Gauss-Seidel / SOR steps over the
 * colours (multiplicative).  The learned source has its own entry point,
 * cs_setup_learned (cascade_learned.h). */
typedef enum { CS_SRC_FROBENIUS = 0, CS_SRC_JACOBI = 1 } cs_source;

/* One level of the geometric hierarchy (Sec. 2.4); levels[0] is the finest and
 * the last level is solved directly.  All pointers are host pointers. */
typedef struct {
    int64_t n;                  /* scalar unknowns on this level */
    int32_t block_size;         /* uniform block size; must divide n */
    const int64_t *a_row_ptr;   /* [n+1] scalar CSR of A_h; column indices sorted per row */
    const int32_t *a_col;       /* [nnz] */
    const double *a_val;        /* [nnz] */
    int64_t n_coarse;           /* unknowns of the next coarser level (0 on the last level) */
    const int64_t *p_row_ptr;   /* [n+1] scalar CSR of the interpolation I_2h^h (n x n_coarse), NULL on the last level */
    const int32_t *p_col;
    const double *p_val;
    double r_scale;             /* restriction R = r_scale * P^T (1 for Galerkin FE/DG, 2^-d for the FD schemes) */
    const int32_t *colour;      /* [n/block_size] block colours 0..chi-1, or NULL (library colours greedily) */
    /* Direct segments: the trailing rows [direct_seg_ptr[0], n) of the level,
     * cut into n_direct_seg independent segments [direct_seg_ptr[k],
     * direct_seg_ptr[k+1]), are solved directly (FP64 dense inverse per
     * segment, at most 8192 rows each) instead of being smoothed and coarsened
     * - the bottom of Alg. 1 for systems that end on this level while others
     * continue.  Rows of a segment couple only with their segment, the other
     * rows never couple to them, and P has no entries in them.  n_direct_seg =
     * 0: no direct rows (the last level is then one segment of all rows). */
    int32_t n_direct_seg;
    const int64_t *direct_seg_ptr;   /* [n_direct_seg+1], increasing, ending at n */
} cs_level;

typedef struct {
    int32_t depth;              /* cascade depth nu >= 1 */
    int32_t mode;               /* cs_mode */
    int32_t order;              /* cs_order */
    int32_t n_pre, n_post;      /* cascade applications before / after the coarse correction (>= 1) */
    int32_t trunc_alpha;        /* keep the alpha largest blocks per row of E (Alg. 2 optional step); 0 = keep all */
    int32_t precision;          /* cs_precision of the V-cycle */
    /* Tikhonov-regularised fit (an extension for reduced-precision cascades,
     * not in the paper): every block solves Lambda~_i (G_i + tau_i I) = H_i with
     * tau_i = ridge * trace(G_i) / n, i.e. it minimises
     * ||E_i - Lambda~_i M_i||_F^2 + tau_i ||Lambda~_i||_F^2 (Alg. 2 least-squares
     * step).  0 = the paper's fit.  Bounds the blocks that cancel nearly
     * dependent directions of M_i, which BF16 application would amplify.
     * Exact fits only (cs_setup, the coarse levels of cs_setup_learned); must
     * be 0 for cs_setup_sketched and for levels with overlapping blocks. */
    double ridge;
    int32_t source;             /* cs_source; cs_setup_sketched and cs_setup_learned take CS_SRC_FROBENIUS only */
    double jacobi_omega;        /* damping of CS_SRC_JACOBI, in (0, 2]; ignored for the fit */
} cs_options;

typedef struct {
    int32_t iterations;         /* V-cycles applied */
    double rel_res;             /* final max_j ||b_j - A x_j||_2 / ||b_j||_2 */
    double rho;                 /* convergence factor from a regression of log residuals (Sec. 3.1) */
    double setup_ms;            /* device time of the last cs_setup */
    double solve_ms;            /* device time of this solve */
    int32_t singular_blocks;    /* blocks solved by the pseudo-inverse fallback in the last setup */
    int32_t precision;          /* cs_precision the solve finished in (raised on divergence) */
    double rho_geo;             /* geometric mean rate (r_K / r_0)^(1/K) over the K iterations */
    double eta;                 /* iterations per decade of residual reduction, log 0.1 / log rho (Sec. 3.1); +inf for rho >= 1 */
} cs_info;

/* Library identity. */
int32_t cs_abi_version(void);
const char *cs_status_string(int32_t status);

/* Create a context on HIP device `device` issuing work on `stream` (a
 * hipStream_t, may be NULL).  *out is set on success. */
cs_status cs_create(cs_ctx *out, int32_t device, void *stream);
void cs_destroy(cs_ctx ctx);
/* Message of the last failing call on ctx (or of the last failed cs_create when ctx is NULL). */
const char *cs_last_error(cs_ctx ctx);

/* Copy the hierarchy to the device.  Validates sizes and column indices;
 * invalidates any previous setup.  The setup checks the diagonals its
 * prescaling needs (CS_EINVAL): a_kk > 0 for elliptic levels (Sec. 2.3.1), a
 * positive viscous diagonal on saddle-point levels (cs_set_saddle_point). */
cs_status cs_set_hierarchy(cs_ctx ctx, int32_t n_levels, const cs_level *levels);

/* Build the cascading smoothers of every level but the last (Alg. 2 /
 * supplementary multicoloured algorithm), the working-precision copies, and the
 * factorisation of the bottom operator.  CS_ECOLOR if a supplied colouring is
 * improper in multiplicative mode; CS_ESINGULAR if a block's normal equations
 * have no positive pivot and the pseudo-inverse fallback fails too. */
cs_status cs_setup(cs_ctx ctx, const cs_options *opt);

/* Change the V-cycle working precision after setup (builds missing copies). */
cs_status cs_set_precision(cs_ctx ctx, int32_t precision);

/* FP64 master smoother Lambda_ell of `level` (ell = 1..depth), unscaled, as host
 * array [n_blocks][block_size][block_size] row-major.  In multiplicative mode
 * block i belongs to Lambda_{ell, colour(i)}.  set_smoother replaces it (and the
 * working-precision copies); the rest of the setup is kept. */
cs_status cs_get_smoother(cs_ctx ctx, int32_t level, int32_t ell, double *blocks_out);
cs_status cs_set_smoother(cs_ctx ctx, int32_t level, int32_t ell, const double *blocks);

/* Structural block pattern of the residual E after fit step `step` of `level`
 * (step 0 = identity; additive: step l = E_l; multiplicative: steps count colour
 * sweeps), as block CSR on the host.  get_pattern_size gives the entry count. */
cs_status cs_get_pattern_size(cs_ctx ctx, int32_t level, int32_t step, int64_t *nnzb);
cs_status cs_get_pattern(cs_ctx ctx, int32_t level, int32_t step, int64_t *row_ptr, int32_t *col);
/* Block colours used on `level` (multiplicative mode), host int32[n_blocks]. */
cs_status cs_get_colours(cs_ctx ctx, int32_t level, int32_t *colours_out);

/* One application of the level's cascade, x <- S(x, b), forward (reverse = 0)
 * or reverse (reverse = 1), in the working precision (Sec. 2.1/2.2/2.4).
 * b, x: device FP64 [n_level][nrhs]. */
cs_status cs_smooth(cs_ctx ctx, int32_t level, int32_t reverse, const double *b, double *x, int32_t nrhs);

/* x = V b: one V-cycle of Algorithm 1 with zero initial guess in the working
 * precision; b, x: device FP64 [n][nrhs] on the finest level. */
cs_status cs_vcycle(cs_ctx ctx, const double *b, double *x, int32_t nrhs);

/* x = V b like cs_vcycle, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, allocation-free
 * harnesses).  The level workspace (x, its double buffer, b and r of every
 * level in the working precision, each range 256-byte aligned: about
 * 4 * sizeof(working type) * nrhs * (total unknowns of all levels) bytes) comes
 * from one static device array of CS_NOALLOC_SCRATCH_MIB MiB per GPU, looked up
 * at cs_create; the call makes no device or host allocation, records no
 * trace events and does not synchronise: x is ready when the context's stream
 * reaches the end of the call.  The kernels are cs_vcycle's, so the result is
 * bit-identical to cs_vcycle's.  Every call on a GPU (any context) shares that
 * GPU's array and leaves its contents behind; calls that overlap on one GPU
 * race.  CS_EINVAL when the workspace would exceed the array or nrhs is not
 * 1, 2, 4 or 8; CS_ESTATE before cs_setup. */
#define CS_NOALLOC_SCRATCH_MIB 64
cs_status cs_vcycle_noalloc(cs_ctx ctx, const double *b, double *x, int32_t nrhs);

/* Solve A x = b by FP64 iterative refinement around the V-cycle: x_0 = 0;
 * r = b - A x (FP64); stop when max_j ||r_j|| <= rtol ||b_j||; x += V r.
 * A residual that becomes non-finite or grows beyond 1e6 ||b|| ends the solve
 * with CS_ENAN; a reduced-precision context then raises its working precision
 * (BF16 -> FP32 -> FP64) for the current setup and solves again.
 * history (host, may be NULL) receives maxit+1 relative residuals.  On
 * CS_ENOCONV x holds the last iterate and info is filled. */
cs_status cs_solve(cs_ctx ctx, const double *b, double *x, int32_t nrhs, double rtol, int32_t maxit,
                   cs_info *info, double *history);

/* Solve A x = b by flexible conjugate gradients with one V-cycle as the
 * preconditioner (the symmetric RF V-cycle of Sec. 2.4 makes it a symmetric
 * preconditioner for SPD A; the flexible form tolerates the working-precision
 * rounding of the V-cycle).  FP64 vectors: x_0 = 0, r = b; per iteration z =
 * V r, p = z + beta p with beta = -(z, A p_prev)/(p_prev, A p_prev), alpha =
 * (p, r)/(p, A p), x += alpha p, r -= alpha A p, each (system, RHS) with its
 * own scalars.  Arguments, stopping test, history and info as for cs_solve;
 * rho is the mean residual reduction per iteration (Sec. 3.1 regression). */
cs_status cs_solve_cg(cs_ctx ctx, const double *b, double *x, int32_t nrhs, double rtol, int32_t maxit,
                      cs_info *info, double *history);

/* Solve A x = b by restarted GMRES(restart) with one V-cycle as the
 * preconditioner: the Sec. 3.1 driver.  FP64 Krylov vectors, the V-cycle in the
 * working precision, independent Krylov spaces per (system, RHS), x_0 = 0.
 *   flexible = 0: left preconditioning (the paper's form); the monitored
 *     residual is ||V (b - A x)||, and the stop is max_j ||V(b_j - A x_j)|| <=
 *     rtol ||V b_j||; history and rho refer to this norm (Sec. 3.1).
 *   flexible = 1: right preconditioning with the preconditioned vectors kept
 *     (flexible GMRES, exact for a V-cycle in reduced precision); the
 *     monitored residual is ||b - A x||, stop as for cs_solve.
 * restart: 1..31 basis vectors per cycle; maxit counts V-cycles inside the
 * Arnoldi steps (the restart checks add one more per cycle).  Memory:
 * (restart + 3) FP64 vectors of n x nrhs (flexible: 2 restart + 3), allocated on
 * the first call and kept.  Errors, history and info as for cs_solve; a
 * diverging reduced-precision V-cycle is escalated the same way. */
cs_status cs_solve_gmres(cs_ctx ctx, const double *b, double *x, int32_t nrhs, double rtol, int32_t maxit,
                         int32_t restart, int32_t flexible, cs_info *info, double *history);

/* Sketched construction (Sec. 4, Concluding Remarks, proposed there): every
 * cascade level is fitted against a tall sketch T = E S of the residual instead
 * of the square E, Lambda~_l = argmin ||(I - Lambda A~) T_{l-1}||_F,
 * T_l = (I - Lambda~_l A~) T_{l-1}, T_0 = S, on the prescaled A~ = W A W, block by
 * block through the same normal equations as cs_setup (multicoloured: colour by
 * colour, Sec. 2.2).  With S = I it reproduces cs_setup.  The memory is 2-3
 * N x s arrays per level instead of the fill-in of E.
 *   S: device FP64, the sketches of all smoothed levels one after the other
 *      (level l: n_l x s, row-major, at offset s * (n_0 + ... + n_{l-1})); the
 *      caller draws them (e.g. Rademacher +-1); only their span matters.
 *   s: sketch width, 1..64, and above the block size when depth > 1 (with
 *      s <= n the first level fits every column exactly, T_1 = 0).
 *   opt: as cs_setup; trunc_alpha must be 0.
 * Residual patterns (cs_get_pattern) are not available after this setup. */
cs_status cs_setup_sketched(cs_ctx ctx, const cs_options *opt, int32_t s, const double *S);

/* Overlapping blocks for `level` (Sec. 3.6.2): n_blocks blocks of m slots
 * (1 <= m <= 16); nodes (host int32[n_blocks][m]) names the unknown of every
 * slot, -1 for an unused slot; every unknown must lie in at least one block
 * (theta = its multiplicity).  The level's cascade becomes
 *   x <- x - diag(theta)^{-1} Theta^T Lambda_l Theta (A x - b),  l = 1..nu,
 * with Lambda_l block-diagonal over the replicated slots, fitted by
 * cs_setup_sketched (additive, FF) against
 *   min ||(Theta - Lambda Theta A~) E_{l-1}||_F,
 *   E_l = diag(theta)^{-1} Theta^T (Theta - Lambda_l Theta A~) E_{l-1}, E_0 = S.
 * cs_get_smoother / cs_set_smoother then move [n_blocks][m][m].  nodes = NULL
 * restores the partition into block rows.  The level must not hold direct
 * segments.  Invalidates the setup. */
cs_status cs_set_overlapping_blocks(cs_ctx ctx, int32_t level, int64_t n_blocks, int32_t m, const int32_t *nodes);

/* Declare `level` a saddle-point (Stokes) level, Sec. 2.3.2: kind (host
 * int32[n_level]) marks every unknown 0 velocity, 1 pressure (constraint row),
 * 2 inert (a decoupled padding unknown; prescaled as a velocity).  The setup
 * then prescales with W = diag(w_u, w_p): w_u so that the prescaled viscous
 * block (the non-pressure columns of the velocity rows) has diagonal
 * ||row||_1 / diagonal, and w_p so that every prescaled constraint row has unit
 * max-norm (l1 = 0) or unit 1-norm (l1 = 1, the staggered-grid variant).  The
 * cascade fit, V-cycle and Krylov drivers are unchanged (the operator is
 * indefinite: use cs_solve_gmres).  kind = NULL restores elliptic prescaling.
 * Call after cs_set_hierarchy; the next setup uses it.  CS_EINVAL for a kind
 * outside 0..2, a level without pressures, and, at setup, a velocity row
 * without a positive diagonal or a pressure row coupled to no velocity. */
cs_status cs_set_saddle_point(cs_ctx ctx, int32_t level, const int32_t *kind, int32_t l1);

/* Stencil-repetition setup cache (Sec. 4, caching the repeated local setups of
 * structured meshes).  coords (host int32[n_blocks][dim], dim 1..3, each
 * coordinate in (-2^28, 2^28), bounding box at most 2^28 points) places every
 * block of `level` at a distinct integer lattice point; the library keeps a
 * copy.  cs_setup then sorts the smoothed blocks into translation classes: at
 * radius r two blocks are equivalent when the lattice translation between them
 * maps every block within r block layers of one onto a block with the same row
 * of A (block-column offsets, stored non-zero values, diagonals of the column
 * blocks).  Cascade step l of a block reads A within l - 1 layers, so only the
 * smallest block of every class at radius l - 1 is fitted; the others copy its
 * Lambda~_l and its residual row E_l with the block columns translated.  The
 * result equals the uncached fit up to the rounding order of the row sums.
 * Used by cs_setup for additive cascades without truncation on elliptic levels
 * without overlapping blocks; elsewhere (and by the sketched and learned
 * setups) every block is fitted.  coords = NULL removes the lattice.
 * CS_EINVAL for a bad dim, coordinates out of range or repeated, or a box too
 * large; at setup, for a residual row above 2048 blocks. */
cs_status cs_set_lattice(cs_ctx ctx, int32_t level, int32_t dim, const int32_t *coords);

/* After an exact setup (cs_setup) of `level`: fitted (host int64[depth]) = the
 * blocks fitted at cascade step l (all smoothed blocks without a lattice);
 * rep (host int32[depth][n_blocks], may be NULL) = the smallest block of every
 * block's translation class at radius l - 1 (each block itself without a
 * lattice).  CS_ESTATE when the last setup of the level was sketched, learned
 * or over overlapping blocks. */
cs_status cs_get_lattice_stats(cs_ctx ctx, int32_t level, int64_t *fitted, int32_t *rep);

/* Pick the launch schedule of every level's cascade sweeps by measurement
 * (needs a setup): for the current working precision and nrhs, one cascade
 * application per level is timed for each candidate schedule (64 or 256 rows
 * per workgroup; a workgroup per tile, or a capped grid of 1024, 2048 or 4096
 * workgroups that loop over the tiles) and the fastest is kept for later
 * solves, until the level is replaced.  Results are identical under every
 * schedule.  Outputs per level (host arrays of n_levels, each may be NULL):
 * rows per workgroup (0 for a level without sweeps), workgroup cap (0 = none)
 * and the best time in ms.  Then one V-cycle is timed eagerly and replayed
 * from a graph, and graph replay of the outer iterations is switched on when
 * it is faster (cs_set_graphs / cs_get_graphs); before that the tail V-cycle's
 * start level is picked the same way (cs_set_tail).  The workspace vectors of
 * every level are overwritten. */
cs_status cs_autotune(cs_ctx ctx, int32_t nrhs, int32_t *wgs, int64_t *grid, double *ms);

/* Graph replay of the outer iterations.  With on = 1, cs_solve and
 * cs_solve_cg issue the device work of every iteration after the first (the
 * V-cycle and the vector updates; the batch's per-system norms included) as
 * one launch of a HIP graph captured on first use, on the context's own
 * stream (ordered after and before the caller's).  The graph is recaptured
 * when the vectors, right-hand-side count, precision, method or device buffers
 * change.  Results are identical to eager launches.  Solves with event
 * tracing on (cs_trace) run eagerly.  cs_autotune decides it by measurement
 * (one V-cycle eager vs replayed); cs_get_graphs reports the setting and, after
 * cs_autotune, both V-cycle times in ms (0 before). */
cs_status cs_set_graphs(cs_ctx ctx, int32_t on);
cs_status cs_get_graphs(cs_ctx ctx, int32_t *on, double *eager_ms, double *graph_ms);

/* Single-workgroup tail V-cycle (Alg. 1 on the small levels).  Levels below a
 * few thousand rows cost a kernel launch per sweep, transfer and direct solve
 * while moving almost no data; from the first level (the finest included) at
 * which every level has at most max_rows rows, the V-cycle from there down is
 * one launch of one workgroup of 512-1024 threads that runs the same per-row
 * arithmetic with workgroup barriers in place of kernel boundaries, so results
 * are bit-identical to the per-level launches.  It applies to additive cascades
 * with fused aggregation transfers, one block size of 1, 2, 4 or 8 on the
 * covered levels, n_pre >= 1 and n_post >= 1; other hierarchies run the
 * per-level launches.  max_rows 0 switches it off (the default).  One
 * workgroup walks a level's 64-row slices one tile after another, so the tail
 * pays only on levels of a few tiles; cs_autotune times one V-cycle with the
 * tail off and starting at each level of at most 65536 rows and keeps the
 * fastest.  cs_vcycle_noalloc always runs the per-level launches.
 * cs_get_tail returns max_rows, the first level the tail covers in the current
 * setup (-1: none) and, when cap > 0, up to cap of the last autotune's
 * candidates (cand_rows: the limit, 0 = off; cand_ms: one V-cycle in ms) with
 * their count in *n_cand (may be null).  Errors: CS_EINVAL for max_rows < 0 or
 * max_rows > 65536. */
cs_status cs_set_tail(cs_ctx ctx, int64_t max_rows);
cs_status cs_get_tail(cs_ctx ctx, int64_t *max_rows, int32_t *first_level, int32_t cap, int64_t *cand_rows,
                      double *cand_ms, int32_t *n_cand);

/* Device timing of kernel classes with HIP events recorded on the context's
 * stream around every launch of the class (for measurement; adds one event pair
 * per recorded launch).  cs_trace(ctx, mask, period) clears the counters and
 * records every period-th launch (period >= 1) of each class whose bit
 * (1 << class) is set in mask; mask 0 stops.  Sampling keeps the event
 * records from perturbing the timed work.  cs_trace_read
 * returns the summed kernel time in ms, the number of launches and the
 * algorithmic bytes those launches must move (structural non-zeros of A with
 * their 32-bit column index, the Lambda blocks, and each vector read or
 * written once). */
typedef enum {
    CS_TRACE_SWEEP = 0,         /* cascade sweeps that read A on large levels (>= 2^19 unknowns) */
    CS_TRACE_SWEEP_ZERO = 1,    /* first sweep from a zero guess: x = Lambda b */
    CS_TRACE_RESIDUAL = 2,      /* residual + restriction, all levels */
    CS_TRACE_PROLONG = 3,       /* interpolation + correction (separate kernel) */
    CS_TRACE_BOTTOM = 4,        /* direct solves: the bottom level and direct segments */
    CS_TRACE_REFINE = 5,        /* FP64 refinement residual and update */
    CS_TRACE_SWEEP_PROLONG = 6, /* first post-sweep with the interpolation fused in */
    CS_TRACE_SWEEP_SMALL = 7,   /* cascade sweeps that read A on small levels */
    CS_TRACE_TAIL = 8,          /* the single-workgroup V-cycle over the coarse levels (cs_set_tail) */
    CS_TRACE_NCLASS = 9
} cs_trace_class;
cs_status cs_trace(cs_ctx ctx, int32_t mask, int32_t period);
cs_status cs_trace_read(cs_ctx ctx, int32_t cls, double *total_ms, int64_t *launches, double *bytes);

/* Streaming reference for the roofline figures above: the HBM rate that plain
 * kernels reach on this device when they only stream arrays (no arithmetic of
 * the method).  Allocates n_read + n_write arrays of `bytes` bytes each on the
 * context's device (freed before returning), fills them, then times `reps`
 * launches on the context's stream that read n_read arrays (0-4) and write
 * n_write (0 or 1) of them, one 16-byte element per thread.  Outputs (host,
 * each may be NULL): *gbps = bytes * (n_read + n_write) / average launch time,
 * in GB/s; *us = the average launch time in microseconds.  Synchronises the
 * device.  Errors: CS_EINVAL for counts out of range, bytes not a positive
 * multiple of 16 or above 64 GiB, reps < 1; CS_ENOMEM when the arrays do not
 * fit in device memory (they come from, and return to, the context's device
 * memory cache). */
cs_status cs_stream_bandwidth(cs_ctx ctx, int32_t n_read, int32_t n_write, int64_t bytes, int32_t reps,
                              double *gbps, double *us);

/* Independent systems sharing one hierarchy (a batch): row_ptr[0..nsys] cuts
 * the finest level into the systems' row ranges (host array, increasing, 0 to
 * n).  cs_solve then measures every (system, right-hand side) residual
 * separately and stops when all of them reach rtol; cs_get_system_stats
 * reports, per system, the V-cycles after which it first converged (or maxit)
 * and its final max relative residual.  nsys = 1 restores one system. */
cs_status cs_set_systems(cs_ctx ctx, int32_t nsys, const int64_t *row_ptr);
cs_status cs_get_system_stats(cs_ctx ctx, int32_t *iterations, double *rel_res);

/* Persist / restore a setup (smoothers, colours, bottom factor) for the same hierarchy. */
cs_status cs_save_setup(cs_ctx ctx, const char *path);
cs_status cs_load_setup(cs_ctx ctx, const char *path);

#ifdef __cplusplus
}
#endif
#endif /* CASCADE_H */
