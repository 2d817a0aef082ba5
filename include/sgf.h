/*
 * sgf.h - C ABI of the Sparse Geometric Factorization (SGF) library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library computes the hierarchical approximate factorization
 *     A ~= A_l = G_1 B_1 G_2 B_2 ... G_l G_l^T ... B_1^T G_1^T
 * of a sparse symmetric positive definite matrix A that comes from a PDE on
 * a Cartesian grid (Klockiewicz & Darve, "Sparse hierarchical
 * preconditioners using piecewise smooth approximations of eigenvectors",
 * Sec. 2.1 and Algorithm 4.1), applies A_l^{-1} (Sec. 4.7) and runs
 * conjugate gradients preconditioned by it (Sec. 7).
 *
 * Conventions shared by every entry point:
 *  - Unknown numbering: grid node (ix, iy[, iz]) has id ix + gx*(iy + gy*iz)
 *    (x fastest); its dofs_per_node unknowns are node*dofs_per_node + comp.
 *  - Return value: SGF_OK or an error code; a thread-local message is kept
 *    for sgf_last_error().  No C++ exception crosses this boundary.  On error
 *    no output handle is created and an existing handle is left usable
 *    unless the code is SGF_EDEVICE.
 *  - Streams: every `stream` argument is a hipStream_t passed as void*
 *    (NULL = the null stream).  Calls enqueue work on that stream; entry
 *    points that return host-visible results (ranks, iteration counts)
 *    synchronize it before returning.
 *  - A handle is not thread safe: use it from one host thread / stream at a
 *    time.  Distinct handles are independent.
 *  - Vectors passed to sgf_apply / sgf_multiply / sgf_pcg_solve are DEVICE
 *    pointers to FP64 column-major n x nrhs arrays owned by the caller.
 */
#ifndef SGF_H
#define SGF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgf_handle_s* sgf_handle;

typedef enum {
  SGF_OK = 0,
  SGF_EINVAL = 1,     /* bad argument, shape or option                      */
  SGF_ENOTSPD = 2,    /* non-positive pivot in a Cholesky (cluster in info) */
  SGF_ENOMEM = 3,     /* device or host allocation failed                    */
  SGF_EDEVICE = 4,    /* HIP runtime error                                   */
  SGF_ENOCONV = 5,    /* CG reached maxit before the tolerance               */
  SGF_ESTATE = 6      /* call out of order (e.g. apply before factorize)     */
} sgf_status;

/* Which cells are compressed, and how (Sec. 5):
 *  SGF_NEST_ALL_ALL  nested-dissection partition; every separator cell but
 *                    single vertices is compressed (Sec. 5.1);
 *  SGF_NEST_2_ALL    only the cells of codimension one (faces in 3D, edges in
 *                    2D);
 *  SGF_NEST_2_2      those cells, with the couplings to the cells on their
 *                    boundary kept exactly: the scaled coupling block of each
 *                    such neighbour enters N whole instead of times its Phi
 *                    (Sec. 5.1), so its span stays in Q_1;
 *  SGF_GEN_ALL_ALL   general partition into boxes of `leaf` vertices per axis
 *                    with no interiors: every box is compressed at every level
 *                    and the compressions are the only eliminations (Sec. 5.2). */
enum { SGF_NEST_ALL_ALL = 0, SGF_NEST_2_ALL = 1, SGF_NEST_2_2 = 2, SGF_GEN_ALL_ALL = 3 };
/* Largest number of columns of a user-supplied near-kernel basis. */
#define SGF_MAX_BASIS_COLS 64
/* When the hierarchy ends (Sec. 4.5 and Sec. 7). */
enum { SGF_STOP_ROOT = 0, SGF_STOP_PAPER = 1 };
/* Arithmetic of the factor and the apply; CG itself is always FP64, and so
 * is the top node's Cholesky.  SGF_FP32_BF16N is SGF_FP32 with the
 * compression matrix N (Eq. 4.5) formed from operands rounded to bfloat16
 * (products accumulated in FP32); N only selects the kept subspace, whose
 * accuracy then drops to about 2^-8, so the default rank threshold of that
 * form is 1e-2. */
enum { SGF_FP64 = 0, SGF_FP32 = 1, SGF_FP32_BF16N = 2 };

typedef struct {
  int32_t dim;                 /* 2 or 3                                           */
  int32_t grid[3];             /* grid nodes per axis (grid[2] ignored in 2D)      */
  int32_t dofs_per_node;       /* 1 (scalar PDE) or 3 (elasticity, Eq. 7.4)        */
  int32_t q;                   /* polynomial degree 0, 1 or 2 (Sec. 3.1)           */
  int32_t leaf;                /* b > 1: level-t period d_t = b * 2^(t-1) (Sec 5.1);
                                  for SGF_GEN_ALL_ALL the level-1 box width      */
  int32_t scheme;              /* SGF_NEST_ALL_ALL (default), SGF_NEST_2_ALL,
                                  SGF_NEST_2_2 or SGF_GEN_ALL_ALL                  */
  int32_t compress;            /* 0 = exact nested-dissection block Cholesky       */
  int32_t compress_from_level; /* first level whose separators are compressed (1) */
  int32_t stop_rule;           /* SGF_STOP_ROOT (default) or SGF_STOP_PAPER        */
  int32_t precision;           /* SGF_FP64 (default), SGF_FP32 or SGF_FP32_BF16N   */
  int32_t tiled_min_rows;      /* levels whose largest front has at least this many
                                  rows are eliminated by the tiled multi-workgroup
                                  path (0: every level, and every compressed
                                  separator's apply uses the multi-workgroup
                                  kernels too); < 0 selects the built-in
                                  threshold.  Fronts that do not fit one
                                  workgroup's LDS panel always take it.           */
  double rank_tol;             /* pivoted-QR rank threshold relative to |R_00|;
                                  <= 0 selects 1e-12 (FP64) / 1e-6 (FP32) /
                                  1e-2 (FP32_BF16N)                              */
} sgf_options;

typedef struct {
  int32_t levels;              /* partitions processed, including the top         */
  int64_t n;                   /* unknowns                                         */
  int64_t top_size;            /* unknowns left for the final exact Cholesky      */
  int64_t factor_entries;      /* stored factor values (L_I, W, L_B, V_B, top)    */
  int64_t factor_bytes;        /* device bytes held by the factor                 */
  int64_t compressed;          /* separators whose rank was below their size      */
  double factor_flops;         /* algorithmic flops of the last numeric factorize */
  double apply_bytes;          /* algorithmic bytes of one apply (factor read 2x) */
  int32_t failed_cluster;      /* cluster id of a non-positive pivot, else -1     */
  int32_t failed_level;        /* its level (1-based), else -1                    */
  int64_t device_bytes;        /* all device memory the handle holds now          */
} sgf_info;

/* Fills *opt with the defaults: scheme NEST_ALL_ALL, compress 1, compress
 * from level 1, stop ROOT, FP64, tiled_min_rows -1 (automatic), rank_tol 0
 * (automatic), q 1, leaf 8. */
void sgf_default_options(sgf_options* opt);

/*
 * Symbolic analysis (Sec. 5.1 partition hierarchy, Algorithm 4.1 REQUIRE):
 * builds the level-1 nodes (nested-dissection cells, interiors then
 * separators), their active sets, the cluster adjacency and all index maps
 * that do not depend on numerical values.
 *   n            number of unknowns = prod(grid) * dofs_per_node
 *   row_ptr      HOST int64[n+1], col_idx HOST int32[nnz]: the FULL
 *                symmetric pattern of A (both triangles), any column order
 *   coords       HOST double[n_nodes * dim], node positions (row per node);
 *                may be NULL when q = 0: the constant needs no geometry
 *                (analyze with q = 0 and no coordinates, then sgf_set_basis,
 *                to use a user basis on a grid without node positions)
 *   opt          options (copied)
 *   out          receives the new handle (caller destroys it)
 * The pattern must only couple nodes within one grid step of each other
 * (the 3^dim vertex stencil assumed in Sec. 5); otherwise SGF_EINVAL.
 * Host-only: no device memory is touched.
 */
sgf_status sgf_analyze(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                       const double* coords, const sgf_options* opt, sgf_handle* out);

/*
 * Numeric factorization (Algorithm 4.1): per level, block-Cholesky of the
 * interiors (Eq. 4.2), polynomial compression of the separators
 * (Eqs. 3.1-3.5, 4.5-4.6), coarsening (Eq. 4.7); exact Cholesky of the
 * last node (Sec. 4.5).
 *   vals         DEVICE double[nnz], values of A in the pattern given to
 *                sgf_analyze (A must be symmetric)
 * May be called again with new values (same pattern): the previous factor
 * is replaced.  Synchronizes `stream` once per level (ranks decide the next
 * level's sizes).  SGF_ENOTSPD when a pivot is not positive.
 */
sgf_status sgf_factorize_numeric(sgf_handle h, const double* vals, void* stream);

/* sgf_analyze followed by sgf_factorize_numeric; `vals` may be a host or a
 * device pointer. */
sgf_status sgf_factorize(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                         const double* vals, const double* coords,
                         const sgf_options* opt, void* stream, sgf_handle* out);

/*
 * Autotuner of the batched elimination (one launch per level over clusters
 * of uneven sizes): factorizes `vals` three times per candidate (trials
 * interleaved) -- the tiled multi-workgroup path, the banded one-wavefront
 * fronts (where the level qualifies) and the one-workgroup-per-front path
 * with panel widths 8, 16 and 32 -- and applies each result once,
 * timing every level's elimination plus `napply` times its forward and
 * backward interior sweeps with device events; each level then keeps the
 * candidate with the fastest of its three times.
 *   vals       DEVICE double[nnz] (as for sgf_factorize_numeric)
 *   napply     weight of the apply (expected applies per factorization)
 *   modes_out  HOST int32[levels] or NULL: chosen candidate per level
 *              (0 tiled, 1 banded one-wavefront fronts, 8/16/32 panel
 *              width, -1 no interiors)
 * Leaves the handle unfactored: call sgf_factorize_numeric next.  The choice
 * persists for later factorizations of the handle.
 */
sgf_status sgf_autotune(sgf_handle h, const double* vals, int32_t napply, int32_t* modes_out,
                        void* stream);

/*
 * z = A_l^{-1} r (Sec. 4.7): forward sweep G_1^{-1}, B_1^{-1}, ..., exact top
 * solve, backward sweep with the transposes.  r and z are DEVICE FP64
 * column-major n x nrhs with leading dimensions ldr, ldz >= n; r == z is
 * allowed.  Does not synchronize.
 */
sgf_status sgf_apply(sgf_handle h, int32_t nrhs, const double* r, int64_t ldr,
                     double* z, int64_t ldz, void* stream);

/*
 * sgf_apply that allocates no device memory, for callers that cannot call
 * hipMalloc: code being captured into a HIP graph, tight serving loops,
 * harnesses that forbid allocation.  Same arguments, kernels and result as
 * sgf_apply (bit for bit); the work vectors (the permuted vector, the
 * separator scratch, the compressed-separator and tiled-front vectors of
 * each level) live in a static device array of SGF_NOALLOC_SCRATCH_BYTES
 * per GPU that the library holds until the process ends, instead of the
 * handle's buffers; every kernel is launched directly (no graph is captured
 * or replayed) and nothing is timed.  Needs n * nrhs * (4 or 8) bytes plus
 * the level vectors to fit: larger requests fail with SGF_EINVAL and a
 * message giving the size.  The array is shared by every handle on a GPU and
 * keeps the last call's contents: calls that overlap on one GPU (other
 * streams or host threads) race and must be serialized by the caller.
 */
#define SGF_NOALLOC_SCRATCH_BYTES (64u << 20)
sgf_status sgf_apply_noalloc(sgf_handle h, int32_t nrhs, const double* r, int64_t ldr,
                             double* z, int64_t ldz, void* stream);

/* y = A_l v (Sec. 2.1 product form; a test hook for the preservation
 * property of Prop. 6.1).  Same layout rules as sgf_apply. */
sgf_status sgf_multiply(sgf_handle h, int32_t nrhs, const double* v, int64_t ldv,
                        double* y, int64_t ldy, void* stream);

/*
 * Conjugate gradients on A x = b preconditioned by A_l^{-1} (Sec. 7): x0 = 0,
 * stop when the recursive residual satisfies ||r_k||_2 / ||b||_2 < rtol.
 * b, x: DEVICE FP64 column-major n x nrhs; each column is an independent CG
 * (per-column scalars, converged columns stop updating).  iters, relres:
 * HOST arrays of nrhs (iterations taken, final recursive relative residual).
 * Returns SGF_ENOCONV if some column did not converge within maxit.
 */
sgf_status sgf_pcg_solve(sgf_handle h, int32_t nrhs, const double* b, int64_t ldb,
                         double* x, int64_t ldx, double rtol, int32_t maxit,
                         int32_t* iters, double* relres, void* stream);

/* y = A v with the CSR matrix held by the handle (FP64).  DEVICE pointers. */
sgf_status sgf_spmv(sgf_handle h, const double* v, double* y, void* stream);

sgf_status sgf_get_info(sgf_handle h, sgf_info* info);

/*
 * Partition export for bit-exact parity checks.
 * sgf_get_perm: HOST int64[n]; perm[slot] = unknown stored in level-1 slot
 *   `slot` (clusters contiguous, ascending cell id; ascending unknown inside).
 * sgf_get_level: for level t (1-based, t <= info.levels) the number of
 *   active clusters (return via *count); when the arrays are non-NULL they
 *   receive, per cluster in ascending cell id: cell id (lexicographic, x
 *   fastest), cell type (number of odd per-axis classes), size of its active
 *   set at the start of the level, and its size after the level's
 *   compressions (= rank when compressed; 0 for eliminated interiors).
 *   Levels above 1 exist only after sgf_factorize_numeric.
 */
sgf_status sgf_get_perm(sgf_handle h, int64_t* perm);
sgf_status sgf_get_level(sgf_handle h, int32_t level, int32_t* count, int32_t* cell_ids,
                         int32_t* types, int32_t* sizes, int32_t* ranks);

/*
 * Factor blocks, for entry-by-entry parity checks of the factorization
 * (Algorithm 4.1).  Level t (1-based) below the top holds, in this order,
 * its interior eliminations (Eq. 4.2; ascending cell id) and then its
 * compressed separators (Eqs. 3.1-3.4; ascending cell id, only those whose
 * rank came out below their size); the top level holds one block, the
 * exact Cholesky factor of what is left (Sec. 4.5).
 * sgf_block_count: the number of blocks of each kind on level t.
 * sgf_export_block: block `index` of level t (eliminations first); fills
 * *info and, for every non-NULL HOST array (column major, FP64 -- converted
 * from FP32 in the FP32 forms):
 *   kind SGF_BLOCK_ELIM: L (m x m, lower, zero above) = chol(M_II) and
 *     W (m x k) = L^{-1} M_IS, the neighbours' unknowns in ascending cell id;
 *   kind SGF_BLOCK_COMP: L (m x m) = chol(M_BB) (Eq. 3.1), V (m x r) the
 *     Householder vectors of the pivoted QR of N (unit diagonal, zero above),
 *     tau (r) their coefficients, Q = H_0 ... H_{r-1} (Eq. 3.3), and rdiag
 *     (r) the diagonal of R;
 *   kind SGF_BLOCK_TOP: L (m x m), the top node's FP64 Cholesky factor.
 * Unused arrays may be NULL.  SGF_ESTATE before a factorization; reads
 * device memory synchronously (the device is synchronized first).
 */
enum { SGF_BLOCK_ELIM = 0, SGF_BLOCK_COMP = 1, SGF_BLOCK_TOP = 2 };
typedef struct {
  int32_t kind;                /* SGF_BLOCK_ELIM / _COMP / _TOP                   */
  int32_t cell;                /* cell id of the cluster (-1 for the top)         */
  int32_t m;                   /* rows of L: interior, separator or top size      */
  int32_t k;                   /* ELIM: columns of W; COMP: neighbour unknowns    */
  int32_t r;                   /* COMP: rank = number of reflectors               */
} sgf_block;
sgf_status sgf_block_count(sgf_handle h, int32_t level, int32_t* n_elim, int32_t* n_comp);
sgf_status sgf_export_block(sgf_handle h, int32_t level, int32_t index, sgf_block* info, double* L,
                            double* W, double* V, double* tau, double* rdiag);

/*
 * Host-only dry run of the level planner, for checking the partition
 * hierarchy without a GPU: replays the coarsening of Sec. 4.3-4.4 with the
 * compression ranks supplied by `rank_fn(level, cell_id, size, ctx)` (called
 * once per compressible separator, level 1-based) instead of computed ones.
 * Afterwards sgf_get_level reports every level.  The handle must not have
 * been factorized; it stays unfactorized (sgf_factorize_numeric re-plans).
 */
typedef int32_t (*sgf_rank_fn)(int32_t level, int64_t cell_id, int32_t size, void* ctx);
sgf_status sgf_plan_dry_run(sgf_handle h, sgf_rank_fn rank_fn, void* ctx);

/*
 * Kernel timing.  While enabled, every kernel launch of the handle is
 * bracketed by two hipEvents recorded on the launch stream, and charged to
 * its kernel class together with the algorithmic work of that launch
 * (flops for the factorization kernels, bytes that must cross HBM for the
 * apply / CG kernels, both from the plan).  sgf_profile_enable(h, 1) clears
 * the counters; sgf_profile_read synchronizes the pending events and copies
 * up to `cap` records (count receives the number of classes).
 */
typedef struct sgf_kernel_stat {
  char name[32];
  int64_t launches;
  double ms;      /* summed event time of the launches                  */
  double flops;   /* summed algorithmic flops                            */
  double bytes;   /* summed algorithmic bytes                            */
} sgf_kernel_stat;
sgf_status sgf_profile_enable(sgf_handle h, int32_t enable);
sgf_status sgf_profile_read(sgf_handle h, sgf_kernel_stat* out, int32_t cap, int32_t* count);
/*
 * Restricts the timing to the launches of one kernel class (the class name
 * as reported by sgf_profile_read, without the "@L<level>" suffix), so that
 * the events bracket only those launches and the rest run as without
 * profiling; NULL or "" times every launch again (the default).  The string
 * is copied.
 */
sgf_status sgf_profile_select(sgf_handle h, const char* kernel_class);

/*
 * Frees every device buffer of the handle (factor, copies of A, work
 * vectors); the symbolic analysis stays, so sgf_factorize_numeric can be
 * called again.  Used to evict a cached factor under a memory budget.
 */
sgf_status sgf_release(sgf_handle h);

/*
 * Device bytes the handle needs to factorize and solve nrhs right-hand
 * sides: for an unfactored handle an upper bound from the plan, every
 * separator at its largest possible rank (min(|B|, columns of N), Sec. 4.5);
 * for a factored one the bytes held plus the work vectors.  Host-only.
 */
sgf_status sgf_estimate_bytes(sgf_handle h, int32_t nrhs, int64_t* bytes);

/*
 * The apply sweep (permutation, all levels' kernels, top) is captured once
 * as a HIP graph on a private stream and replayed on the caller's stream
 * while its arguments (nrhs, r, ldr, z, ldz) and the factorization stay the
 * same -- as they do inside sgf_pcg_solve.  enable = 0 launches every kernel
 * directly (per-kernel profiling needs this) and keeps the captured graph
 * for when it is enabled again; default 1.
 */
sgf_status sgf_set_apply_graph(sgf_handle h, int32_t enable);

/*
 * Launch shape of the per-level work lists of the one-workgroup elimination
 * and of the compression (one launch per level over clusters of uneven
 * size).  0 (default): one workgroup per cluster, in cluster order.
 * max_workgroups > 0: persistent launches on at most that many workgroups,
 * which take clusters from a counter, costliest first when the costs differ
 * by more than 2x.  Results do not depend on the launch shape.
 */
sgf_status sgf_set_persistent(sgf_handle h, int32_t max_workgroups);

/*
 * Elimination (Eq. 4.2) of levels whose interiors all have M_II of lower
 * bandwidth below 32 and at most 64 separator rows: enable = 1 (default)
 * runs one wavefront per front (band Cholesky in LDS, L_SI row by row in
 * registers, L_SI L_SI^T on the matrix cores), one launch per group of
 * fronts of equal ring width (8, 16, 24, 32); 0 uses the panel kernels.
 * Same factor up to rounding order.  Takes effect at the next factorization.
 */
sgf_status sgf_set_band_elim(sgf_handle h, int32_t enable);

/*
 * Compression (Eqs. 3.1-3.4) of levels whose separators all have at most 64
 * rows and at most 128 columns of N: enable = 1 (default) runs each separator
 * with its front, Phi blocks and N staged in LDS, on four wavefronts when the
 * level has fewer than 1024 separators of at most 32 rows (wavefront 0 alone
 * in the Cholesky and the pivoted QR) and on one otherwise; 2 the same on one
 * wavefront at every level (the same values as 1, bit for bit); 0 uses the
 * one-workgroup kernel (also used under sgf_set_persistent).  Same ranks and,
 * up to rounding order, the same factor.  Takes effect at the next
 * factorization.
 */
sgf_status sgf_set_small_compress(sgf_handle h, int32_t enable);

/*
 * Coarsening into the next level (Secs. 4.3-4.4): enable = 1 (default) has
 * the copy kernel compute every block's destination from the structure of
 * the two levels and the sizes after the compressions (per-separator father
 * and offset from the host); 0 builds the copy list of every block on the
 * host instead.  The same copies, so the same factor bit for bit.  Re-plans
 * and drops the factor.
 */
sgf_status sgf_set_device_coarsen(sgf_handle h, int32_t enable);

/*
 * Kernel of the coarse couplings C_ab = T_a M_ab T_b^T of the pairs that
 * touch a compressed separator (Sec. 3.2): mode 0 one workgroup per pair
 * (its intermediate product in device scratch), 1 one wavefront per pair
 * (four per workgroup, the intermediate in LDS) whenever that fits, -1
 * (default) the wavefront kernel on levels with at least 4096 such pairs.
 * Both form the same products in the same order (the same bits).  Takes
 * effect at the next factorization.
 */
sgf_status sgf_set_pair_kernel(sgf_handle h, int32_t mode);

/*
 * Interior sweeps of the apply (Sec. 4.7) on levels whose M_II blocks have a
 * lower bandwidth of at most 64: enable = 1 (default) stages the band of L_I
 * in LDS and solves it one wavefront per right-hand side, and with a single
 * right-hand side on a level of the banded elimination gives each front's
 * band solve one wavefront (x and the band in registers, the coefficients in
 * an LDS tile) and its L_SI products a workgroup; these are the operations of
 * mode 2 in the same order, so the same values (a zero product can only turn
 * a -0 into +0).  2 keeps the banded sweeps but one workgroup per front for
 * every right-hand-side count; 0 uses the blocked sweeps that also serve
 * dense interiors.  All give the same result up to rounding order.  Drops a
 * captured apply graph.
 */
sgf_status sgf_set_band_apply(sgf_handle h, int32_t enable);

/*
 * Interior sweeps of the apply (Sec. 4.7) with one right-hand side on levels
 * whose interiors all have at most 64 rows (the upper levels of a 2D grid):
 * enable = 1 (default) gives each front one workgroup that issues every load
 * of the front before waiting and solves with a single wavefront; 0 uses the
 * blocked sweeps.  Same result up to rounding order.  Drops a captured apply
 * graph.  SGF_EINVAL for a NULL handle or another value.
 */
sgf_status sgf_set_small_apply(sgf_handle h, int32_t enable);

/*
 * User-supplied near-kernel basis (Secs. 1 and 3.1: the method needs a
 * partition hierarchy and a matrix Pi whose columns span the near kernel,
 * e.g. rigid-body modes, not necessarily monomials of the coordinates):
 * Phi_B = Pi(B, :) for every level-1 node.
 *   ncols   1..SGF_MAX_BASIS_COLS columns; 0 returns to the monomials of
 *           degree q (which need the coordinates unless q = 0)
 *   basis   HOST double[n * ncols], column major (entry (i, p) at
 *           basis[i + p * n], i the unknown id), finite; copied
 * Re-plans level 1 and drops the factor (call sgf_factorize_numeric next);
 * also ends the low-rank mode.  SGF_EINVAL on a bad size or value.
 */
sgf_status sgf_set_basis(sgf_handle h, int32_t ncols, const double* basis);

/*
 * The standard low-rank equivalent of the compression (Sec. 7.4, Eq. 7.5),
 * for comparison with the polynomial one: each separator B is compressed
 * with Q taken from the pivoted QR of its scaled off-diagonal block
 * [Mhat_BX1 | Mhat_BX2 | ...] (no L_B^T Phi_B block), cut after exactly the
 * rank that the polynomial compression found for B.
 *   enable = 1  records the ranks of the handle's current (polynomial)
 *               factorization, per level and separator, and uses them for the
 *               next factorizations (SGF_ESTATE if the handle is not
 *               factored); the levels keep the sizes they had, so the
 *               factorization has the same structure;
 *   enable = 0  returns to the polynomial compression.
 * Re-plans level 1 and drops the factor; call sgf_factorize_numeric next
 * (with the same values to compare the two at equal ranks).  Same pivot, tie
 * and reflector conventions as the polynomial QR; a step whose trailing
 * part is zero keeps its column and takes no reflection.
 */
sgf_status sgf_set_low_rank(sgf_handle h, int32_t enable);

/* Releases every host and device resource of the handle (NULL is a no-op). */
sgf_status sgf_destroy(sgf_handle h);

const char* sgf_status_str(sgf_status s);
const char* sgf_last_error(void);

/* ------------------------------------------------------------------------
 * Serving loop (continuous batching of many operators on one GPU)
 * ------------------------------------------------------------------------
 * Operators are registered once (analysis on the host); requests to solve
 * nrhs right-hand sides with an operator -- factorizing it first when its
 * factor is not on the device or when asked to -- are queued and started by
 * `slots` worker threads, each with its own HIP stream, as soon as a slot
 * and device memory are free.  Memory: the bytes the factors hold plus the
 * bytes reserved for running requests stay within hbm_budget; cached factors
 * that are not in use are evicted least-recently-used (sgf_release) to make
 * room.  Waiting solves of one operator are coalesced into one
 * multi-right-hand-side PCG of up to max_batch_rhs columns; columns are
 * independent, so each result equals the result of the request alone.
 * Threading: submit / wait may be called from any thread. */
typedef struct sgf_server_s* sgf_server;

typedef struct {
  int64_t hbm_budget;          /* device bytes for factors + running requests   */
  int32_t slots;               /* concurrent requests (worker streams), 1..16    */
  int32_t max_batch_rhs;       /* columns of one coalesced PCG, 1..256          */
} sgf_server_options;

typedef struct {
  int64_t ticket;
  int32_t op;
  int32_t nrhs;
  int32_t status;              /* sgf_status of the request                       */
  int32_t factorized;          /* 1 if its batch factorized the operator         */
  int32_t batch_rhs;           /* columns of the PCG it ran in                    */
  int32_t slot;                /* worker that ran it                              */
  int32_t iters_max;           /* largest CG iteration count of its columns      */
  double relres_max;           /* largest final relative residual                */
  double t_submit, t_start, t_end;   /* sgf_server_clock() seconds            */
  double t_factor;             /* seconds spent factorizing in its batch         */
} sgf_request_info;

typedef struct {
  int64_t held_bytes;          /* device bytes held by cached factors             */
  int64_t peak_bytes;          /* largest held + reserved seen                    */
  int64_t evictions, factorizations, batches, queued, cached_operators;
} sgf_server_stats;

/* Defaults: 200 GiB budget, 4 slots, 16 columns per batch. */
void sgf_server_default_options(sgf_server_options* opt);
/* With the environment variable SGF_SERVER_TRACE set at creation, every
 * finished batch prints one bookkeeping line (slot, operator, columns, bytes
 * reserved, held before and after, totals) on stderr. */
sgf_status sgf_server_create(const sgf_server_options* opt, sgf_server* out);
/* Registers an operator: the arguments of sgf_analyze plus its values
 * (HOST double[nnz]); all are copied.  Its analysis runs on a worker, ahead
 * of its first request (a failing analysis fails that operator's requests
 * with its status).  *op_id receives its id. */
sgf_status sgf_server_add_operator(sgf_server s, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                                   const double* vals, const double* coords, const sgf_options* opt,
                                   int32_t* op_id);
/* Queues a request: b, x DEVICE double (n x nrhs, leading dims ldb, ldx),
 * borrowed until the request completes; refactor != 0 factorizes even if a
 * factor is cached.  nrhs <= max_batch_rhs.  *ticket identifies it. */
sgf_status sgf_server_submit(sgf_server s, int32_t op_id, int32_t refactor, int32_t nrhs, const double* b,
                             int64_t ldb, double* x, int64_t ldx, double rtol, int32_t maxit, int64_t* ticket);
/* Blocks until the request is done; fills info and, if not NULL, the HOST
 * arrays iters[nrhs] and relres[nrhs].  A ticket can be waited for once.
 * A request whose memory need exceeds the whole budget ends with status
 * SGF_ENOMEM. */
sgf_status sgf_server_wait(sgf_server s, int64_t ticket, sgf_request_info* info, int32_t* iters,
                           double* relres);
sgf_status sgf_server_get_stats(sgf_server s, sgf_server_stats* out);
/* The clock of the t_* fields (monotonic seconds). */
double sgf_server_clock(void);
/* Finishes every queued request, stops the workers, destroys the operators. */
sgf_status sgf_server_destroy(sgf_server s);

#ifdef __cplusplus
}
#endif

#endif /* SGF_H */
