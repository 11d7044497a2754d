/* d3m.h -- C ABI of the D3M dual factorization and solution library for
 * AMD MI355X (gfx950).
 *
 * What it computes (Sec. II of Moshfegh, Makris, Vouvakis, "Parallel Direct
 * Domain Decomposition Methods (D3M) for Finite Elements", 2019): the
 * reduced matrix K of D3M is block-wise sparse; its dense blocks couple the
 * interfaces between domains (Fig. 1(b)).  The dual step factors K with a
 * block LDL^T -- per nonzero block a dense factorization, dense triangular
 * solves and dense updates, arranged as a task DAG built by simulating the
 * sequential algorithm (Sec. II, Fig. 1(c)) -- and then solves with the
 * factors.  Here K is complex symmetric (K = K^T, transposes are never
 * conjugated), factored without pivoting as P K P^T = L D L^T with L unit
 * lower triangular and D diagonal, P the block permutation of the
 * elimination order (nested dissection over the domain grid, or a given
 * order).
 *
 * Layouts (all complex numbers interleaved re,im; "c128" = 2 x double):
 *   K     one flat device buffer: for each interface I (user numbering) the
 *         full n_I x n_I diagonal block, column-major, of which only the
 *         lower triangle is read; then for each pair (I,J), I > J, in the
 *         order given to d3m_analyze, the n_I x n_J block K_IJ, column-major.
 *         K_JI = K_IJ^T is implied.  Offsets: d3m_plan_k_offsets.
 *   B, X  nrhs right-hand sides / solutions, RHS j at ptr + j*ld, each an
 *         N-vector in user row numbering (rows of interface 0 first).
 *   dK    same layout as K (full diagonal blocks are written).
 *
 * Ownership: the caller owns every device buffer (K, B, X, G, Lambda, dK and
 * the workspace).  The library allocates no device memory: everything it
 * needs lives in the workspace handed to d3m_factor_bind.  K must stay alive
 * and unchanged between d3m_factorize and the last d3m_solve/d3m_adjoint,
 * because refinement residuals read it.  Plans and factors own host memory
 * only and free it in their destroy calls.
 *
 * Errors: negative codes are caller or runtime errors and are detected on
 * the host before anything is enqueued.  Positive codes are numerical
 * outcomes written by the device and reported by d3m_status_sync (LAPACK
 * info style); they never abort the stream.
 *
 * Streams: factorize/solve/adjoint/batch_run enqueue on the given stream and
 * neither allocate, synchronize nor call back to the host (unless
 * d3m_options.ir_host_sync is set), so they can be captured in a hipGraph.
 * Calls on one factor must not overlap in time.
 */
#ifndef D3M_H
#define D3M_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct d3m_plan_s* d3m_plan;     /* host symbolic: pattern, order, fill, DAG */
typedef struct d3m_factor_s* d3m_factor; /* numeric factor bound to a workspace      */
typedef struct d3m_batch_s* d3m_batch;   /* many factors, one persistent launch      */
typedef void* d3m_stream;                /* a hipStream_t (NULL = default stream)    */

typedef enum {
  D3M_OK = 0,
  D3M_ERR_ARG = -1,       /* null handle, bad size, bad pointer                      */
  D3M_ERR_PATTERN = -2,   /* duplicate/self/out-of-range pair, order not a permutation */
  D3M_ERR_WORKSPACE = -3, /* workspace too small or misaligned                        */
  D3M_ERR_STATE = -4,     /* call out of sequence (solve before factorize, ...)       */
  D3M_ERR_HIP = -5,       /* a HIP runtime call failed                                */
  D3M_ERR_HANG = -6,      /* a dependency wait exceeded the watchdog bound           */
  D3M_ERR_NORUNTIME = -7, /* no usable gfx950 device                                  */
  D3M_ZERO_PIVOT = 1,     /* a pivot d_k was zero or not finite (row in run_info)     */
  D3M_NONFINITE = 2,      /* a non-finite value in the solution or residual          */
  D3M_IR_NOCONV = 3       /* refinement did not reach the tolerance                  */
} d3m_status;

typedef enum {
  D3M_C128 = 0,   /* complex128 factor and solve                                    */
  D3M_C64_IR = 1  /* complex64 factor (FP32 MFMA, FP32 accumulation) + FP64 refinement */
} d3m_precision;

/* Analysis options.  Zero-initialise for defaults. */
typedef struct {
  int32_t tile;      /* largest tile edge, a multiple of 16 in [16,128]; 0 -> 128 */
  int32_t nworkers;  /* persistent workgroups assumed by the list scheduler; 0 -> 256 */
  int32_t sched;     /* 0 = list scheduling by bottom level, 1 = plain sequential order */
  int32_t nelim;     /* 0: eliminate every block.  > 0: a partial elimination for the
                        primal reduction (d3m_reduce / d3m_recover): only the first nelim
                        blocks of the order are eliminated; the others must be the user ids
                        0..nred-1 (nred = nblk - nelim), the pairs between them must come
                        first in the pair list, and eliminating the first nelim blocks must
                                                fill no block between them that is not such a pair */
  int32_t solve_tile; /* rows of a solve task, a multiple of 16 in [16,128]; 0 -> 64 */
  int32_t merge;      /* source panels per merged Schur update task, [1,16]; 0 -> 8 */
  int32_t rhs_groups; /* also build a solve DAG that splits the right-hand sides into this
                         many column groups (independent copies, twice the parallelism at two
                         groups); used by solves with >= 16 columns per group.  [1,8]; 0 -> 1 */
  int32_t reserved;
} d3m_analyze_options;

/* Numeric options.  Zero-initialise for defaults. */
typedef struct {
  double tol;           /* refinement target on eta_inf; 0 -> 1e-10                  */
  int32_t max_iter;     /* refinement steps after x0; 0 -> 10                         */
  int32_t ir_host_sync; /* 1: read eta back after every step and stop exactly        */
  double growth_dmin;   /* FP32 fallback trigger: min|d| < growth_dmin * max|A_II|; 0 -> 1e-4 */
  double growth_lmax;   /* FP32 fallback trigger: max|L| > growth_lmax; 0 -> 1e2      */
  int32_t fallback;     /* 1 (default via 0): re-factor tripped blocks in FP64; -1 off */
  int32_t timing;       /* 1: record HIP events around every DAG launch (run_info times) */
  int32_t dk_stored;    /* 1: d3m_adjoint returns dK with respect to the stored entries of
                           the K buffer: a stored off-diagonal entry also moves its mirror
                           (x2), a diagonal block is read from its lower triangle (strict
                           lower x2, diagonal x1, upper 0); 0: the symmetric block gradient */
  int32_t pivot;        /* 1: Bunch-Kaufman pivoting (1x1 and 2x2 pivots, the sytrf of Sec. II)
                           inside each diagonal tile of at most `tile` unknowns; the block
                           pattern and the task DAG are unchanged.  No FP64 re-factoring of
                           tiles then.  0: no pivoting (the stated method) */
} d3m_options;

typedef struct {
  int64_t N;            /* unknowns                                                  */
  int64_t nblk, npair;  /* interfaces, stored off-diagonal blocks                       */
  int64_t k_len;        /* complex elements of the K buffer                            */
  int64_t fill_blocks;  /* blocks of L created by elimination                           */
  int64_t L_blocks;     /* off-diagonal blocks of L                                     */
  int64_t nnz_L;        /* lower-triangle entries of L (diagonal blocks counted as lower triangles) */
  int64_t nnz_K;        /* lower-triangle entries of K                                  */
  int64_t etree_height, max_S;
  int64_t ntask_factor, ntask_solve, ntiles;
  double flops_diag, flops_trsm, flops_update, flops_factor; /* 8 real flops per complex FMA */
  double solve_flops_per_rhs;                                /* 16 * nnz_L                  */
  double sim_factor_us; /* list-scheduler estimate of the factor makespan                 */
} d3m_plan_info;

typedef struct {
  int32_t status;       /* a d3m_status                                              */
  int32_t ir_iters;     /* refinement steps taken (0 for the FP64 path)               */
  int64_t pivot_row;    /* user row of the first bad pivot, or -1                     */
  double eta;           /* final max-over-columns normwise backward error             */
  double eta_hist[32];  /* eta after x0 and after each refinement step                */
  int32_t fallbacks;    /* diagonal blocks re-factored in FP64                        */
  int32_t hang;         /* watchdog fired                                             */
  /* with d3m_options.timing: HIP-event time of the persistent DAG launches
   * since the previous d3m_status_sync (summed), and their counts */
  double t_factor_dag_ms, t_solve_dag_ms;
  int32_t n_factor_dag, n_solve_dag;
  double knorm;         /* ||K||_inf (max row sum of |k_ij|) of the last factorized K  */
} d3m_run_info;

/* Build the symbolic plan.
 *   nblk, blk_size   interface count and sizes (all >= 1)
 *   npair, pairs     2*npair ids, unordered, I != J, each pair once
 *   order            nblk ids, the elimination order, or NULL
 *   grid             3 ints (domain grid a x b x c whose interfaces, numbered
 *                    axis 0 first then 1 then 2, lower domain x slowest, are
 *                    the nblk interfaces) or NULL.  With order == NULL and a
 *                    grid: nested dissection over the grid; with neither:
 *                    greedy minimum degree on the block graph.
 * The DAG of Sec. II (Fig. 1(c)) is built here by simulating the sequential
 * elimination; tasks are ordered by a list scheduler (bottom-level priority). */
d3m_status d3m_analyze(int32_t nblk, const int32_t* blk_size, int64_t npair, const int32_t* pairs,
                       const int32_t* order, const int32_t* grid, const d3m_analyze_options* opt,
                       d3m_plan* out);
d3m_status d3m_plan_query(d3m_plan plan, d3m_plan_info* out);
/* The elimination order (nblk user ids). */
d3m_status d3m_plan_order(d3m_plan plan, int32_t* order);
/* nblk + npair + 1 offsets (complex elements) of the K blocks. */
d3m_status d3m_plan_k_offsets(d3m_plan plan, int64_t* offsets);
/* S_I (later neighbours after fill, in elimination order) of user interface I;
 * writes at most nblk ids and returns the count in *count. */
d3m_status d3m_plan_struct(d3m_plan plan, int32_t I, int32_t* S, int32_t* count);
/* Static check of the DAG on the CPU: every storage tile's writers are
 * totally ordered and every reader is ordered after the writer it needs.
 * Only for small plans (quadratic memory in the task count). */
d3m_status d3m_plan_check(d3m_plan plan, int64_t* nviolations);
void d3m_plan_destroy(d3m_plan plan);

/* Workspace for one factor with up to nrhs_max right-hand sides per solve. */
d3m_status d3m_workspace_bytes(d3m_plan plan, d3m_precision prec, int32_t nrhs_max, size_t* bytes);
/* Bind a factor to a caller-owned device workspace (256-byte aligned) and
 * upload its task tables (synchronous; not on the hot path). */
d3m_status d3m_factor_bind(d3m_plan plan, d3m_precision prec, void* dev_ws, size_t bytes,
                           int32_t nrhs_max, const d3m_options* opt, d3m_factor* out);
/* Factor K (c128 layout above) on the stream: scatter/convert, then one
 * persistent launch of the elimination DAG -- Sec. II, the dual
 * factorization: per nonzero block of K a dense factorization of the
 * diagonal block (the sytrf-like LDL^T, here without pivoting), dense
 * triangular solves (triSolve) of the blocks below it and dense updates
 * (GEMM) of the blocks it reaches, ordered by the task graph of Fig. 1(c).
 * Numerical outcomes (a zero or non-finite pivot) go to d3m_status_sync. */
d3m_status d3m_factorize(d3m_factor f, const void* dev_K, d3m_stream stream);
/* X = K^{-1} B for nrhs <= nrhs_max columns -- Sec. II, the dual solution
 * with the factors (block forward, diagonal and backward solves).
 * D3M_C128: FP64 solve plus one certifying FP64 residual.  D3M_C64_IR (not
 * in the paper; classical mixed-precision iterative refinement): FP32 solves
 * with FP64 residuals r = B - K X on the original K and FP64 updates until
 * the normwise backward error eta_inf = ||r||/(||K|| ||x|| + ||b||) of every
 * column is <= tol.  B and X are caller device buffers (layout above, may
 * not overlap); errors as for every call. */
d3m_status d3m_solve(d3m_factor f, const void* dev_K, const void* dev_B, void* dev_X,
                     int32_t nrhs, int64_t ld, d3m_stream stream);
/* Adjoint with the same factors.  Not in the paper (which differentiates
 * nothing): it is the adjoint of the linear solve x = K^{-1} b.  For a real
 * objective J(x), dJ/db = K^{-T} G = K^{-1} G because K = K^T, so the solve
 * above yields Lambda = K^{-1} G with no second factorization, and
 * dJ/dK = -Lambda X^T restricted to K's block pattern and symmetrized:
 * dK = -sym(Lambda X^T), sym(A) = (A + A^T)/2, summed over columns
 * (holomorphic convention: for J = sum_k Re(c_k^T x_k) pass G = C).  With
 * d3m_options.dk_stored the values are weighted per stored entry instead.
 * X is the solution of the forward solve; dK (K's layout) may be NULL. */
d3m_status d3m_adjoint(d3m_factor f, const void* dev_K, const void* dev_X, const void* dev_G,
                       void* dev_Lambda, void* dev_dK, int32_t nrhs, int64_t ld, d3m_stream stream);
/* Primal reduction (Sec. II, the first part of the task graph: per domain
 * the factorization of the regularized domain matrix and its map onto its
 * interfaces, assembled into the reduced matrix).  The factor's plan is a
 * partial elimination (d3m_analyze_options.nelim) of a primal matrix A in
 * block form, given in the K layout of that plan: the eliminated blocks are
 * the domains' interior unknowns, the blocks left (user ids 0..nred-1) the
 * interfaces.  Computes, with a complex128 factor:
 *   Kred = A_GG - A_Gi A_ii^-1 A_iG   (the Schur complement on the blocks
 *          left, written whole in the K layout of those blocks and of the
 *          first npair_red pairs; may be NULL),
 *   Gred = F_G - A_Gi A_ii^-1 F_i     (nrhs columns, ldg >= their rows;
 *          with F == NULL nothing is solved and d3m_recover cannot follow).
 * F: nrhs <= nrhs_max primal right-hand sides (ldf >= N).  Kred, Gred are
 * then the input of an ordinary factor of the reduced matrix.  Numerical
 * outcomes (a zero pivot of an interior block) go to d3m_status_sync. */
d3m_status d3m_reduce(d3m_factor f, const void* dev_A, const void* dev_F, int64_t ldf, void* dev_Kred,
                      void* dev_Gred, int64_t ldg, int32_t nrhs, d3m_stream stream);
/* Primal recovery (Sec. II, the third part: per domain the recovery of the
 * primal unknowns and, optionally, the scattering matrix S).  After
 * d3m_reduce with the same nrhs and the solution Xred of the reduced system
 * (ldx >= its rows): U = the full primal solution, the interior unknowns
 * u_i = A_ii^-1 (F_i - A_iG Xred) and Xred itself in the rows of the blocks
 * left (ldu >= N).  With nports > 0 also S (nports x nrhs, column-major),
 * S_pq = sum_r M(r, p) U(r, q), bilinear, for the port modes M (N x nports,
 * ldm >= N). */
d3m_status d3m_recover(d3m_factor f, const void* dev_Xred, int64_t ldx, void* dev_U, int64_t ldu, int32_t nrhs,
                       const void* dev_M, int64_t ldm, int32_t nports, void* dev_S, d3m_stream stream);
/* Wait for the factor's last stream and report numerical outcomes, in the
 * manner of LAPACK's info argument (not from the paper): the first bad
 * pivot's user row, refinement steps and eta, FP64 re-factors, DAG times. */
d3m_status d3m_status_sync(d3m_factor f, d3m_run_info* out);
/* Copy one factor block to host memory as c128, column-major: (J == I) the
 * diagonal block of I (L strictly below the diagonal, D on it), otherwise
 * L_JI (n_J x n_I) for J in S_I.  Synchronous; for tests and inspection. */
d3m_status d3m_factor_block(d3m_factor f, int32_t J, int32_t I, void* host_out);
/* With d3m_options.pivot: the interchanges of user interface I after
 * d3m_factorize -- perm[i] (n_I) is the original index inside I of the
 * unknown at position i (each diagonal tile permuted inside itself) -- and
 * D's off-diagonal entries as c128 (doff[i] = D(i+1, i) when a 2x2 pivot
 * starts at i, else 0).  Synchronous; for tests and inspection.  The factor
 * blocks (d3m_factor_block) hold the factor in LAPACK's product form: rows
 * of a tile in columns left of it keep their original order, and a 2x2
 * pivot at i keeps D(i+1, i) in the slot of L(i+1, i), which is zero. */
d3m_status d3m_factor_pivots(d3m_factor f, int32_t I, int32_t* perm, void* doff_host);
/* Diagnostics: record, for every ticket of the following DAG launches, four
 * int64 values {taken, dependencies met, done, workgroup} (times on the
 * device's 100 MHz constant clock) into dev_buf: factor launches in the
 * first half, solve launches in the second half (each half must hold
 * 32 bytes per task, else that DAG is not traced).  NULL stops tracing. */
d3m_status d3m_factor_set_trace(d3m_factor f, void* dev_buf, size_t bytes);
/* Task list of the factor (solve = 0) or solve (1) DAG in ticket order:
 * kinds, panels (elimination position) and m,n,k triples; NULL arrays
 * query the count only. */
d3m_status d3m_factor_tasks(d3m_factor f, int32_t solve, int32_t* kinds, int32_t* panels, int32_t* mnk,
                            int32_t* count);
void d3m_factor_destroy(d3m_factor f);

/* Batching: many bound factors (their own plans and workspaces) run as one
 * persistent launch per phase -- the task graphs of independent problems
 * (a frequency sweep) merged and list-scheduled together, as Sec. II
 * schedules one weighted B-DAG onto the processors.  The batch keeps its
 * merged task tables in dev_ws (size from d3m_batch_workspace_bytes). */
d3m_status d3m_batch_workspace_bytes(int32_t ninst, const d3m_factor* f, size_t* bytes);
d3m_status d3m_batch_create(int32_t ninst, const d3m_factor* f, void* dev_ws, size_t bytes,
                            d3m_batch* out);
/* Factor and solve every instance: K[i], B[i], X[i] with nrhs[i] columns and
 * leading dimension ld[i]. */
d3m_status d3m_batch_run(d3m_batch b, const void* const* K, const void* const* B, void* const* X,
                         const int32_t* nrhs, const int64_t* ld, d3m_stream stream);
void d3m_batch_destroy(d3m_batch b);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, serving loops, harnesses that forbid hipMalloc): d3m_factor_bind
 * on a device array of the library itself instead of a caller workspace.
 * The array holds D3M_STATIC_WS_BYTES per device (each device the library is
 * loaded on keeps it until the process ends); a plan whose workspace
 * (d3m_workspace_bytes) is larger returns D3M_ERR_WORKSPACE.  No device
 * memory is allocated here or by the factor's later calls.  One factor per
 * device lives in the array: binding another one on the same device
 * invalidates the earlier (its calls then return D3M_ERR_STATE), and calls
 * on factors that share the array must not overlap in time (they race).
 * d3m_options.timing is ignored.  Bind on the device that will run it
 * (the current device). */
#define D3M_STATIC_WS_BYTES (64u << 20)
d3m_status d3m_factor_bind_static(d3m_plan plan, d3m_precision prec, int32_t nrhs_max, const d3m_options* opt,
                                  d3m_factor* out);

/* Engine measurement (the benchmarked GEMM weight of the paper's Sec. II
 * scheduling, measured on this device): times the task-body GEMM on every
 * workgroup of the device along each candidate load path, for the
 * precision, and writes each candidate's aggregate GFLOP/s (8 flops per
 * complex multiply-add) to gflops_out[0 .. *ncand - 1] (*ncand = 4):
 *   0  update tile 128x128x512, the factor's path (direct global->LDS loads
 *      for complex64, register slabs for complex128);
 *   1  update tile through register slabs of half the depth;
 *   2  solve tile 64x64x448 (right-hand-side block shared by all
 *      workgroups), whole k per wave;
 *   3  the solve tile with k split over two wave halves, the solve's path.
 * *best_id is the faster of the update-tile candidates 0 and 1.
 * dev_scratch: device memory of at least 256*3*128*512 complex elements of
 * the precision (overwritten); D3M_ERR_WORKSPACE if bytes is smaller.
 * Synchronizes the device. */
d3m_status d3m_tune_gemm(d3m_precision prec, void* dev_scratch, size_t bytes, int32_t* best_id,
                         double* gflops_out /* [ncand] or NULL */, int32_t* ncand);

/* Diagnostics: one tile product of the library's MFMA engine on device data,
 *   C(i,j) = alpha * sum_p A(i,p) d(p) B(j,p) + beta * C(i,j),
 * i < m <= 128, j < n <= 128, p < k; complex128 (prec D3M_C128) or complex64
 * (D3M_C64_IR) operands.  amode 0: A(i,p) = A[i + p*lda]; 1: A[i*lda + p];
 * 2: symmetric block read from its lower triangle, A(i,p) = S(i0+i, p).
 * B(j,p) = B[j + p*ldb]; C(i,j) = C[i + j*ldc]; d may be NULL.  Runs on
 * the stream; for unit tests of the engine. */
d3m_status d3m_debug_gemm(d3m_precision prec, int32_t m, int32_t n, int32_t k, int32_t amode, int32_t i0,
                          const void* A, int64_t lda, const void* d, const void* B, int64_t ldb, void* C,
                          int64_t ldc, double alpha, double beta, d3m_stream stream);

const char* d3m_status_string(d3m_status s);
/* 1 if the library was built with gfx950 device code and a device is present. */
int32_t d3m_device_ok(void);

#ifdef __cplusplus
}
#endif
#endif /* D3M_H */
