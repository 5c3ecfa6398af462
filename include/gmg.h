/*
 * gmg.h - C ABI of the MI355X (gfx950) Gravo MG setup + solve library.
 *
 * Method: Wiersma, Nasikun, Eisemann & Hildebrandt, "A Fast Geometric
 * Multigrid Method for Curved Surfaces" (SIGGRAPH 2023).  The library builds
 * the multigrid hierarchy of Sec. 4 (sampling, graph Voronoi cells,
 * Voronoi-neighbour triangles, barycentric prolongation) and the Galerkin
 * operators of Alg. 1, then solves A x = b with the V-cycle of Alg. 2.
 *
 * Conventions for every call:
 *  - Arrays named *_dev are device pointers on the current HIP device; arrays
 *    named *_host are host pointers.  Indices are int32, values float64.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *    All device work is enqueued on it.
 *  - Return value: GMG_OK (0), GMG_NOT_CONVERGED (+1, a warning), or a
 *    negative error code.  gmg_last_error() gives a message for the calling
 *    thread's last failure.
 *  - Levels are numbered from 0 (the input points, the paper's level 1) to
 *    num_levels - 1 (the coarsest level, solved directly).
 */
#ifndef GMG_H
#define GMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum gmg_status {
  GMG_OK = 0,
  GMG_NOT_CONVERGED = 1,      /* max_iters reached; x holds the last iterate */
  GMG_INVALID_ARGUMENT = -1,  /* null pointer, bad size, out-of-range/unsorted index, non-finite value */
  GMG_OUT_OF_MEMORY = -2,
  GMG_DEVICE_ERROR = -3,      /* a HIP runtime failure */
  GMG_NOT_SPD = -4,           /* non-positive diagonal at some level or non-positive Cholesky pivot */
  GMG_DEGENERATE = -5         /* coarsening stalled with a coarsest level too large to factor densely */
};

typedef struct gmg_handle_s* gmg_handle;

/* Options of the hierarchy construction and V-cycle.  struct_size must equal
 * sizeof(gmg_options); gmg_default_options() fills the paper's settings. */
typedef struct gmg_options {
  int32_t struct_size;
  double coarsening_ratio;       /* phi of Eq. (1): keep about phi of the points per level (1/8) */
  int32_t min_coarse_points;     /* coarsen while a level has more points than this (1000, Sec. 4.2) */
  int32_t max_levels;            /* upper bound on the number of levels (32) */
  int32_t nu_pre, nu_post;       /* Gauss-Seidel sweeps before/after the coarse correction (2, 2; Sec. 5.1) */
  int32_t shift_coarse_points;   /* 1: move coarse points to their Voronoi-cell mean (Sec. 4.4) */
  int32_t sample_order;          /* 0: hashed sweep order (default), 1: input index order (Sec. 4.2) */
  uint64_t seed;                 /* seed of the hashed sweep and colouring orders */
  int32_t weighting;             /* prolongation weights on the chosen triangle: 0 barycentric (Sec. 4.4,
                                    default), 1 uniform, 2 inverse distance (the variants of the
                                    weighting ablation, Sec. 5.3) */
  int32_t fallback_on_vertex;    /* 1: also use the inverse-distance fallback when the closest point of
                                    the best triangle is one of its vertices (default 0: edge and
                                    vertex projections are kept, Sec. 4.4) */
  int32_t color_passes;          /* iterated-greedy recolouring passes after the first-fit colouring that
                                    orders the multicolour Gauss-Seidel sweeps (3; 0 keeps the first
                                    colouring; at most 64) */
  int32_t block_min_rows;        /* levels 1.. (not the coarsest) with more points than this sweep in block
                                    order (4096): the points, projected onto the two coordinate axes of
                                    largest extent, are binned into square cells slightly wider than the
                                    longest coupling of A_l along those axes; the four parity classes of
                                    the cells are swept one after the other, and within a cell the
                                    colours in order.  A valid Gauss-Seidel order (the paper leaves the
                                    order open, Sec. 3) that needs four launches per sweep. */
  int32_t autotune;              /* 1 (default): the lanes per row of the row kernels of every level solved by
                                    separate launches, and the load chunk of level 0's, are picked by timing
                                    the candidates on the level's data at the build (cached per shape class
                                    for the process; a shape never changes a result bit); 0: fixed rules */
} gmg_options;

/* Values of gmg_options.weighting. */
enum gmg_weighting { GMG_WEIGHTS_BARYCENTRIC = 0, GMG_WEIGHTS_UNIFORM = 1, GMG_WEIGHTS_INVERSE_DISTANCE = 2 };

typedef struct gmg_solve_info {
  int32_t iterations;            /* V-cycles performed */
  int32_t converged;             /* 1 if ||b - A x|| <= tol ||b|| */
  double rel_residual;           /* ||b - A x||_2 / ||b||_2 after the last V-cycle */
} gmg_solve_info;

/* Fills *o with the defaults listed above.  Returns GMG_INVALID_ARGUMENT if o is NULL. */
int gmg_default_options(gmg_options* o);

/*
 * Builds the hierarchy (Sec. 4 and Alg. 1): levels are coarsened while they
 * have more than min_coarse_points points; every level gets its prolongation
 * P_l (at most 3 entries per row), its Galerkin operator A_{l+1} = P_l^T A_l
 * P_l and a Gauss-Seidel colouring; the coarsest level gets a dense Cholesky
 * factorisation.
 *
 *  n            number of points (> 0)
 *  points_dev   n x 3 row-major float64 positions
 *  m            number of input edges (>= 0)
 *  edges_dev    m x 2 int32 point pairs; any order, duplicates and self loops allowed
 *  A_rowptr_dev, A_col_dev, A_val_dev, A_nnz
 *               the n x n system matrix in CSR: rowptr[0] = 0, rowptr[n] = A_nnz,
 *               strictly ascending columns per row, symmetric pattern that
 *               contains the diagonal, finite values, positive diagonal
 *  opt          options (NULL: defaults)
 *  stream       hipStream_t; the call returns after the stream has finished the build
 *  out          receives the handle (NULL on error)
 *
 * The library copies what it keeps; the caller may free the inputs on return.
 * The handle owns all device memory of the hierarchy until gmg_free().
 * Errors: GMG_INVALID_ARGUMENT, GMG_NOT_SPD, GMG_DEGENERATE, GMG_OUT_OF_MEMORY,
 * GMG_DEVICE_ERROR.
 */
int gmg_build_hierarchy(int64_t n, const double* points_dev, int64_t m, const int32_t* edges_dev,
                        const int32_t* A_rowptr_dev, const int32_t* A_col_dev,
                        const double* A_val_dev, int64_t A_nnz, const gmg_options* opt,
                        void* stream, gmg_handle* out);

/*
 * Solves A x = b (Alg. 1): repeats V-cycles (Alg. 2) from the initial guess
 * in x_dev until ||b - A x||_2 <= tol ||b||_2 or max_iters cycles were run.
 *
 *  b_dev, x_dev       float64 device vectors of length n (x_dev: in = initial guess, out = solution)
 *  tol                relative tolerance (>= 0)
 *  max_iters          maximum number of V-cycles (>= 1)
 *  info               optional host struct receiving iterations / converged / rel_residual
 *  residual_history   optional host array of max_iters doubles: relative residual after each cycle
 *
 * If b = 0 the solution x = 0 is returned after 0 cycles.  Synchronises the
 * stream once per V-cycle (convergence test).  One solve at a time per handle.
 * Returns GMG_OK, GMG_NOT_CONVERGED, GMG_INVALID_ARGUMENT or GMG_DEVICE_ERROR.
 */
int gmg_solve(gmg_handle h, const double* b_dev, double* x_dev, double tol, int32_t max_iters,
              void* stream, gmg_solve_info* info, double* residual_history);

/*
 * gmg_solve_pcg for nrhs right-hand sides on one hierarchy, processed in
 * groups of 8 that share every launch: each matrix entry read serves the 8
 * right-hand sides of a group, and the latency of each V-cycle phase is paid
 * once per group.  Each right-hand side gets the arithmetic of gmg_solve_pcg
 * except the order in which its dot products are summed.
 *
 *  B_dev, X_dev   float64 device arrays of nrhs x n values, right-hand side / solution q
 *                 contiguous at offset q * n (X_dev: in = initial guesses, out = solutions)
 *  infos          host array of nrhs gmg_solve_info: for right-hand side q the first
 *                 iteration at which it met tol, converged, and its true relative residual
 *  tol, max_iters, precision, stream: as for gmg_solve_pcg; a group iterates until all of its
 *                 right-hand sides have converged (b = 0 gives x = 0)
 * Returns GMG_OK, GMG_NOT_CONVERGED (some right-hand side missed tol), GMG_INVALID_ARGUMENT,
 * GMG_NOT_SPD, GMG_OUT_OF_MEMORY or GMG_DEVICE_ERROR.
 */
int gmg_solve_pcg_batched(gmg_handle h, int32_t nrhs, const double* B_dev, double* X_dev, double tol,
                          int32_t max_iters, int32_t precision, void* stream, gmg_solve_info* infos);

/*
 * gmg_solve_pcg_batched for a group of hierarchies at once (many meshes, many
 * right-hand sides; Sec. 2 and Sec. 5.5 motivate many solves per hierarchy):
 * every step of a CG iteration is one launch for all members still
 * iterating, so the launch latency is paid once per group instead of once per
 * mesh, and the whole iteration is one replayed hipGraph.  Member m runs
 * exactly the steps of gmg_solve_pcg_batched on its own hierarchy, so its
 * solutions, iteration counts and residuals are bit-identical to a
 * gmg_solve_pcg_batched call with the same arguments; members that have
 * converged stop while the others go on.
 *
 *  count          number of members (>= 0)
 *  handles        host array of count distinct handles on one device
 *  nrhs           host array: member m's right-hand sides, 0..8 (0: member skipped)
 *  B_dev, X_dev   host arrays of count device pointers, each laid out as in
 *                 gmg_solve_pcg_batched for its member (X: initial guesses in, solutions out)
 *  tol, max_iters, precision, stream: as for gmg_solve_pcg_batched (every member's
 *                 work is queued on `stream`, which is synchronised on return)
 *  infos          host array of count x 8 gmg_solve_info: member m's right-hand side q at
 *                 m * 8 + q (entries q >= nrhs[m] untouched)
 *  status_out     host array of count statuses (GMG_OK or GMG_NOT_CONVERGED per member)
 * Returns GMG_OK if every member converged, GMG_NOT_CONVERGED if some did not,
 * GMG_INVALID_ARGUMENT (repeated handle, handles on different devices, nrhs
 * outside 0..8, null pointers, non-finite B or X), GMG_NOT_SPD,
 * GMG_OUT_OF_MEMORY or GMG_DEVICE_ERROR.  A handle of the group must not be
 * used by another call until this one returns.
 */
int gmg_solve_pcg_grouped(int32_t count, const gmg_handle* handles, const int32_t* nrhs, const double* const* B_dev,
                          double* const* X_dev, double tol, int32_t max_iters, int32_t precision, void* stream,
                          gmg_solve_info* infos, int32_t* status_out);

/*
 * gmg_precondition for nrhs vectors (layout as in gmg_solve_pcg_batched):
 * Z_q = B R_q, one symmetric V-cycle from zero per vector.
 */
int gmg_precondition_batched(gmg_handle h, int32_t nrhs, const double* R_dev, double* Z_dev, int32_t precision,
                             void* stream);

/*
 * Replaces the values of A (same sparsity pattern as at the build) and
 * recomputes what depends on them: the Galerkin operators A_l of every
 * coarser level (Alg. 1), their solve layouts and the factorisation of the
 * coarsest one.  The hierarchy itself (samples, Voronoi cells, P_l,
 * colourings) is geometric and is kept: a geometric hierarchy only has to be
 * rebuilt when the domain changes (Sec. 2), as in the applications whose
 * matrix changes from solve to solve (Sec. 5.5).
 *
 *  A_val_dev   float64 device array of the handle's nnz(A_1) values, in the CSR order given to
 *              gmg_build_hierarchy; finite, positive diagonal
 *  stream      hipStream_t; returns after the stream has finished
 *
 * Returns GMG_OK, GMG_INVALID_ARGUMENT, GMG_NOT_SPD (non-positive diagonal or coarse
 * pivot) or GMG_DEVICE_ERROR.  After an error the handle's operators are undefined until
 * a successful update; gmg_free stays valid.
 */
int gmg_update_matrix(gmg_handle h, const double* A_val_dev, void* stream);

/*
 * out[e] = scale * u_i * v_j for every stored entry e = (i, j) of an n x n CSR
 * pattern.  With u = lambda (the adjoint solution of A lambda = dL/dx, A
 * symmetric), v = x and scale = -1 this is dL/dA on A's pattern for a loss L
 * of the solution of A x = b (and dL/db = lambda).
 *
 *  n                  rows; rowptr_dev int32[n+1], col_dev int32[nnz] (device)
 *  u_dev, v_dev       float64 device vectors of length n
 *  out_dev            float64 device array of nnz values (written)
 *  stream             hipStream_t (asynchronous; no synchronisation)
 * Returns GMG_OK, GMG_INVALID_ARGUMENT or GMG_DEVICE_ERROR (launch failure).
 */
int gmg_pattern_outer(int64_t n, const int32_t* rowptr_dev, const int32_t* col_dev, const double* u_dev,
                      const double* v_dev, double scale, double* out_dev, void* stream);

/* Precision of the V-cycle used as a CG preconditioner. */
enum gmg_precision {
  GMG_PRECISION_F64 = 0, /* the cycle in double */
  GMG_PRECISION_F32 = 1  /* float copies of A_l, P_l and the iterates; coarsest solve in double */
};

/*
 * Solves A x = b by conjugate gradients in double precision, preconditioned
 * by one symmetric V-cycle per iteration: the method used as the
 * preconditioner of a Krylov solver, the extension the paper names in its
 * conclusion (Sec. 6), with the hierarchy of Sec. 4 and the cycle of Alg. 2
 * (smoothing before the coarse correction visits the colours in ascending
 * order, after it in descending order, so the cycle from a zero guess is a
 * symmetric operator).
 *
 *  b_dev, x_dev       float64 device vectors of length n (x_dev: in = initial guess, out = solution)
 *  tol                relative tolerance (>= 0) on ||b - A x||_2 / ||b||_2
 *  max_iters          maximum number of CG iterations (>= 1)
 *  precision          GMG_PRECISION_F64 or GMG_PRECISION_F32: arithmetic of the cycle.  The
 *                     residual, the solution update, every dot product and the coarsest
 *                     (dense Cholesky) solve stay in double.
 *  info               optional: iterations, converged, and the TRUE relative residual at exit
 *  residual_history   optional host array of max_iters doubles: the recursively updated
 *                     relative residual after each iteration
 *
 * The CG form is the flexible one (Polak-Ribiere coefficient), which stays a
 * conjugate-direction method when the float cycle carries rounding.  When the
 * recursive residual passes the test the true residual is computed; if that
 * one does not pass, it replaces the recursive one and the iteration goes on.
 * Float copies of the level data are made on the first F32 call (about
 * 4 bytes per matrix entry) and kept by the handle.  Synchronises the stream
 * once per iteration.  One solve at a time per handle.
 * Returns GMG_OK, GMG_NOT_CONVERGED, GMG_INVALID_ARGUMENT, GMG_NOT_SPD (non-positive
 * curvature: A or the cycle is not positive definite), GMG_OUT_OF_MEMORY or GMG_DEVICE_ERROR.
 */
int gmg_solve_pcg(gmg_handle h, const double* b_dev, double* x_dev, double tol, int32_t max_iters,
                  int32_t precision, void* stream, gmg_solve_info* info, double* residual_history);

/*
 * z = B r: one symmetric V-cycle (the CG preconditioner above) from a zero
 * guess, in the given precision.  r_dev, z_dev: float64 device vectors of
 * length n (may not alias).  For callers with their own Krylov method.
 * Returns GMG_OK, GMG_INVALID_ARGUMENT (also for non-finite r), GMG_OUT_OF_MEMORY
 * or GMG_DEVICE_ERROR; the call returns after the stream has finished.
 */
int gmg_precondition(gmg_handle h, const double* r_dev, double* z_dev, int32_t precision, void* stream);

/*
 * gmg_precondition without allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same z = B r, same kernels and the same bits as
 * gmg_precondition; the residual in the solve numbering and the cycle's
 * level-0 output live in a fixed device array of the library (32 MiB per
 * device, held until the process ends), so the call allocates nothing, does
 * not synchronise and does not check r for non-finite values (a non-finite r
 * gives a non-finite z).
 *
 *  h                  a handle of the current device with at most 2,097,152 points
 *  r_dev, z_dev       float64 device vectors of length n (may not alias)
 *  precision          GMG_PRECISION_F64, or GMG_PRECISION_F32 once the handle holds its float
 *                     level data (made by its first F32 call of gmg_precondition or gmg_solve_pcg)
 *  stream             the work is enqueued on it; z is ready when the stream reaches that point
 *
 * Every call on a device shares that device's array, which keeps the last
 * call's contents: calls that overlap on one device race, and so do
 * overlapping calls on one handle.
 * Returns GMG_OK, GMG_INVALID_ARGUMENT (bad arguments, too many points, float data not made yet,
 * another device current) or GMG_DEVICE_ERROR (a launch failed).
 */
int gmg_precondition_noalloc(gmg_handle h, const double* r_dev, double* z_dev, int32_t precision, void* stream);

/* Releases the handle and its device memory.  NULL is ignored. */
void gmg_free(gmg_handle h);

/* Static text for a status code. */
const char* gmg_status_string(int status);

/* Message of the calling thread's last failing call ("" if none). */
const char* gmg_last_error(void);

/* Number of levels of the hierarchy. */
int gmg_num_levels(gmg_handle h, int32_t* levels);

/*
 * Sizes of level l, written to sizes_host[0..8]:
 *  0 points n_l, 1 undirected edges of E_l, 2 nnz(A_l), 3 nnz(P_l) (0 on the
 *  coarsest level), 4 colours, 5 rows of P_l that used the inverse-distance
 *  fallback, 6 coarse points sampled from this level (0 on the coarsest),
 *  7 entries of the symmetric edge CSR (2 x edges), 8 one if the level's
 *  Gauss-Seidel sweeps run in block order (see gmg_options.block_min_rows).
 */
int gmg_level_sizes(gmg_handle h, int32_t level, int64_t* sizes_host);

/*
 * The row-kernel shapes level l's V-cycle uses, written to out_host[0..4]:
 *  0 lanes per row of the row kernels of A_l (residual, colour sweeps; levels >= 1 solved by
 *    separate launches, else 0), 1 lanes per row of the restriction by P_l^T (1: one lane per row;
 *    levels solved by separate launches, else 0), 2 entries per load chunk of level 0's row kernels (level 0, else 0),
 *  3 one if the level's sweeps run as block sweeps (one workgroup per grid cell, four launches),
 *  4 the uniform slice width level 0's row kernels use (its SELL padded to the longest row, chosen
 *    where that stores at most 1.15 times the entries and measures faster; else 0).
 */
int gmg_level_tuning(gmg_handle h, int32_t level, int32_t* out_host);

/* Export codes of gmg_export_level (element type and count for level l). */
enum gmg_export_what {
  GMG_EXPORT_POSITIONS = 0,    /* double[n*3] points of the level */
  GMG_EXPORT_EDGE_ROWPTR = 1,  /* int32[n+1] symmetric edge CSR */
  GMG_EXPORT_EDGE_COL = 2,     /* int32[2m] neighbours, ascending per row */
  GMG_EXPORT_EDGE_W = 3,       /* double[2m] Euclidean edge lengths */
  GMG_EXPORT_SCALARS = 4,      /* double[2] mean edge length e_hat and sampling radius r */
  GMG_EXPORT_SAMPLES = 5,      /* int32[n_{l+1}] points kept as coarse points, ascending */
  GMG_EXPORT_LABELS = 6,       /* int32[n] coarse point (Voronoi cell) of each point */
  GMG_EXPORT_DIST = 7,         /* double[n] graph distance to the cell's coarse point */
  GMG_EXPORT_P_COL = 8,        /* int32[3n] prolongation columns, row-major, unused = -1 */
  GMG_EXPORT_P_VAL = 9,        /* double[3n] prolongation weights, unused = 0 */
  GMG_EXPORT_P_CNT = 10,       /* int32[n] entries per row of P_l */
  GMG_EXPORT_TRI = 11,         /* int32[2n] chosen triangle (j, k) with apex label(p); -1 = fallback */
  GMG_EXPORT_A_ROWPTR = 12,    /* int32[n+1] CSR of A_l */
  GMG_EXPORT_A_COL = 13,       /* int32[nnz] */
  GMG_EXPORT_A_VAL = 14,       /* double[nnz] */
  GMG_EXPORT_COLORS = 15,      /* int32[n] Gauss-Seidel colour of each row */
  GMG_EXPORT_CHOL = 16,        /* double[n*n] row-major lower Cholesky factor (coarsest level only) */
  GMG_EXPORT_COARSE_INVERSE = 17, /* double[n*n] inverse of the coarsest A by columns: element k*n + i is
                                    (A^-1 e_k)_i (coarsest level only; the direct solve of Alg. 2 is the
                                    product with it, summed over k ascending) */
  GMG_EXPORT_BLOCK_COLORS = 18 /* int32[n] block colour of each point (0..2 for bricks of two grid cells,
                                  0..3 for single cells), on levels swept in block order; size 0 elsewhere */
};

/*
 * Copies one array of level l to host memory (inspection and testing).
 * `bytes` must equal the array's size exactly; otherwise GMG_INVALID_ARGUMENT.
 * Arrays a level does not have (e.g. LABELS on the coarsest level) have size 0.
 */
int gmg_export_level(gmg_handle h, int32_t level, int32_t what, void* host_dst, int64_t bytes);

/*
 * Measurement support (not part of the method).  Times every launch of one
 * kernel class with a pair of HIP events recorded on the stream that kernel is
 * launched on, and accumulates the algorithmic bytes of those launches
 * (12 bytes per matrix entry read, 28 per row: right-hand side, diagonal,
 * row length, result).  Process-wide: one timing session at a time.
 *
 *  kernel              GMG_TIMER_GS_FINEST: one colour of a Gauss-Seidel sweep on level 0;
 *                      GMG_TIMER_RESIDUAL_FINEST: residual + norm partials on level 0;
 *                      GMG_TIMER_GS_GALERKIN: one colour of a sweep on a Galerkin level
 *                      (solved by separate launches, i.e. above the single-workgroup tail)
 *  expected_launches   events to pre-create (more are created on demand)
 * The timed launches of a solve are issued directly instead of from its
 * captured graph.  gmg_timer_stop waits for the recorded events and returns
 * the summed kernel time in milliseconds, the number of timed launches and
 * their bytes.
 */
enum gmg_timer_kernel { GMG_TIMER_GS_FINEST = 0, GMG_TIMER_RESIDUAL_FINEST = 1, GMG_TIMER_GS_GALERKIN = 2 };
int gmg_timer_start(int32_t kernel, int32_t expected_launches);
int gmg_timer_stop(double* total_ms, int64_t* launches, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* GMG_H */
