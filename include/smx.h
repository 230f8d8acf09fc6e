/*
 * smx.h - C ABI of libsmx: density matrices of a block-sparse, symmetric,
 * orthogonalised Kohn-Sham matrix by the submatrix method with a
 * Newton-Schulz matrix-sign iteration, on one AMD Instinct MI355X (gfx950).
 *
 * The operation (Lass, Schade, Kuehne, Plessl, "A Submatrix-Based Method for
 * Approximate Matrix Function Evaluation in the Quantum Chemistry Code
 * CP2K"):
 *
 *   For every group g of block columns of K (Sec. III-A overview applied per
 *   block column, Sec. IV-C; several block columns may be combined into one
 *   submatrix, Sec. IV-C "Generating Submatrices From Multiple Block
 *   Columns"):
 *     1. R(g) = the block rows stored in any column of g (ascending);
 *        A_g = K[R(g), R(g)] - mu I, unstored blocks taken as zero.
 *     2. S_g = sign(A_g) (Eq. sign / signev), evaluated by the second-order
 *        Newton-Schulz iteration X_{k+1} = X_k (3I - X_k^2) / 2 (Sec. II-B)
 *        from X_0 = A_g / s_g, where s_g = ||A_g||_inf is a Gershgorin bound
 *        on the spectral radius; stopped when max|X_k^2 - I| <= tol.
 *     3. The group's own block columns of D_g = (I - S_g) / 2 (Eq. DsignSym
 *        with S = I) are written into D, only at the block positions stored
 *        in K (the result keeps K's sparsity pattern).
 *   Then N = Tr D (Sec. IV-G, no spin factor) and E = Tr(D K) (Eq.
 *   bandenergy), reduced in FP64.
 *
 * Conventions
 *   - Every function returns an int32_t status: SMX_OK (0) or a negative
 *     SMX_E_* code.  Nothing throws across the ABI.  smx_last_error() gives a
 *     message for the last failing call on a context.
 *   - A context is not thread-safe; use one per host thread.
 *   - Input arrays are borrowed for the duration of the call only and are
 *     copied.  Outputs go to caller-owned buffers.  The context owns its
 *     device memory and frees it in smx_destroy().
 *   - Device work is enqueued on the stream given to smx_set_stream() (the
 *     null stream by default), e.g. the current PyTorch stream.  Functions
 *     that return host scalars synchronise that stream.
 *
 * Block-sparse layout (BSC, "block compressed sparse column"):
 *   nblk block rows/columns with sizes blk_size[0..nblk-1] (1..1024);
 *   block column J holds storage positions col_ptr[J] .. col_ptr[J+1]-1
 *   (col_ptr int64, col_ptr[0] = 0), whose block rows row_idx[p] ascend
 *   strictly.  BOTH triangles are stored and every diagonal block must be
 *   present.  Block (I, J) is a dense column-major blk_size[I] x
 *   blk_size[J] array at the running offset of all preceding blocks in
 *   storage order, so values has sum_p blk_size[row_idx[p]] *
 *   blk_size[col(p)] doubles.  D is returned in exactly the same layout.
 */
#ifndef SMX_H
#define SMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SMX_OK                 0
#define SMX_E_INVALID         -1   /* bad argument, size or layout            */
#define SMX_E_STATE           -2   /* call order (e.g. evaluate before load)  */
#define SMX_E_NOT_SYMMETRIC   -3   /* |K_IJ - K_JI^T| > 1e-12 max|K|          */
#define SMX_E_NONFINITE       -4   /* NaN/Inf in K or in an iterate           */
#define SMX_E_UNSUPPORTED     -5   /* option not implemented on this path     */
#define SMX_E_NOMEM           -6   /* device or host allocation failed        */
#define SMX_E_HIP             -7   /* HIP runtime error                        */
#define SMX_E_NOT_CONVERGED   -8   /* a group did not converge; D is written  */

/* ---- precision modes (smx_set_precision) ------------------------------- */
#define SMX_FP64      0   /* every Newton-Schulz product in FP64 (MFMA f64)      */
#define SMX_BF16_3W   1   /* bulk products as 3-word BF16 splits (6 MFMA bf16
                             products, FP32 accumulation), then FP64 polish     */
#define SMX_BF16_1W   2   /* bulk products in plain BF16 (FP32 accumulation),
                             then FP64 polish                                    */
#define SMX_FP32      3   /* bulk products in FP32 (MFMA f32 16x16x4, FP32
                             accumulation), then FP64 polish                    */
#define SMX_FP16_2W   4   /* bulk products as 2-word FP16 splits (3 MFMA f16
                             products, FP32 accumulation), then FP64 polish     */

/* ---- solvers (smx_set_solver) --------------------------------------------- */
#define SMX_SOLVER_ITERATIVE 0   /* sign by Newton-Schulz / Pade products (kT = 0 only) */
#define SMX_SOLVER_EIG       1   /* diagonalisation of every submatrix (Sec. IV-F)     */

/* ---- sign iterations (smx_set_iteration) --------------------------------- */
#define SMX_ITER_NS2    0   /* second-order Newton-Schulz X (3I - X^2) / 2 (Sec. II-B)   */
#define SMX_ITER_PADE3  1   /* third-order Pade X (15I - 10X^2 + 3X^4) / 8 (Sec. VI-A) */

typedef struct smx_context *smx_ctx;

typedef struct {
    int32_t ngroups;          /* number of submatrices                            */
    int32_t n_min, n_max;     /* min / max submatrix dimension n_g                */
    int32_t iters_min, iters_max;  /* Newton-Schulz iterations per group (bulk +
                                      polish), i.e. the k at which X_k was taken   */
    int32_t n_not_converged;  /* groups that hit max_iter                         */
    int32_t precision;        /* precision mode of the last evaluation            */
    int32_t nwaves;           /* waves the groups were processed in (see
                                 smx_set_workspace_limit)                          */
    double  n_mean;           /* mean n_g                                         */
    double  iters_mean;
    double  resid_max;        /* max over groups of the last computed max|X^2 - I| */
    double  algo_flops;       /* sum_g 2 n_g^3 x dense products: two per Newton-
                                 Schulz step, three per Pade step                  */
    double  exec_flops;       /* flops issued to the matrix cores (padding, half
                                 tiles and multi-word products included)           */
    double  time_gather_ms;   /* device time of the last evaluation, per phase    */
    double  time_iterate_ms;
    double  time_scatter_ms;
    double  time_total_ms;
    double  workspace_bytes;  /* device memory held by the context                */
} smx_stats;

/* Lifetime.  `device` is a HIP device ordinal; the context makes it current
 * in every call. */
int32_t smx_create(int32_t device, smx_ctx *out);
int32_t smx_destroy(smx_ctx ctx);

/* Message for the last failing call on ctx (never NULL; valid until the next
 * call on ctx).  smx_last_error(NULL) describes the last smx_create failure. */
const char *smx_last_error(smx_ctx ctx);

/* Enqueue all device work on `hip_stream` (a hipStream_t; NULL = null stream). */
int32_t smx_set_stream(smx_ctx ctx, void *hip_stream);

/*
 * Load K (Sec. II-C: DBCSR-style dense blocks with a sparse block index).
 * blk_size, col_ptr and row_idx are host arrays; `values` is a host pointer,
 * or a device pointer when values_on_device != 0.  Validates the layout
 * (SMX_E_INVALID), finiteness (SMX_E_NONFINITE) and symmetry
 * max|K_IJ - K_JI^T| <= 1e-12 max|K| (SMX_E_NOT_SYMMETRIC).  Resets the
 * groups to one group per block column and invalidates any result.
 */
int32_t smx_load_k(smx_ctx ctx, int32_t nblk, const int32_t *blk_size,
                   const int64_t *col_ptr, const int32_t *row_idx,
                   const double *values, int32_t values_on_device);

/*
 * Replace K's values, keeping the pattern of the last smx_load_k (the plan
 * is reused).  Same validation of values as smx_load_k.
 */
int32_t smx_update_values(smx_ctx ctx, const double *values, int32_t values_on_device);

/*
 * Partition the block columns into submatrix groups (Sec. IV-C): group g
 * owns block columns grp_blocks[grp_ptr[g] .. grp_ptr[g+1]-1].  Every block
 * column must appear in exactly one group (else SMX_E_INVALID).  Host arrays.
 */
int32_t smx_set_groups(smx_ctx ctx, int32_t ngroups, const int32_t *grp_ptr,
                       const int32_t *grp_blocks);

/* Chemical potential mu (Hartree) of D = (I - sign(K - mu I)) / 2. */
int32_t smx_set_mu(smx_ctx ctx, double mu);

/* Electronic temperature kT in Hartree.  kT = 0: D = (I - sign(K - mu I)) / 2.
 * kT > 0: D_g = Q f(Lambda) Q^T with the Fermi function f(x) = 1 / (1 +
 * exp(x / kT)) of the eigenvalues of K_sub - mu I (Sec. IV-F); the
 * evaluation then diagonalises every submatrix (see smx_set_solver). */
int32_t smx_set_temperature(smx_ctx ctx, double kT);

/*
 * Solver of the submatrix function.  SMX_SOLVER_ITERATIVE (default): the
 * sign by matrix products (smx_set_iteration, smx_set_precision); needs
 * kT = 0.  SMX_SOLVER_EIG: diagonalisation of every submatrix, the paper's
 * production path (Sec. IV-F), at any kT, in FP64: Householder reduction to
 * tridiagonal form (one workgroup per submatrix), eigenvalues by bisection on
 * Sturm counts, eigenvectors by twisted factorisations (clusters of
 * eigenvalues closer than 1e-8 ||T|| by inverse iteration with
 * orthogonalisation), then only the own columns of D, as
 * Q diag(f) Q^T E through thin products.  At kT = 0 an eigenvalue with
 * |lambda - mu| <= 1e-14 ||A_g||_inf gets weight 1/2 (Eq. signevext).  kT > 0
 * always uses this path.  Limit: n_g <= 3072 (SMX_E_UNSUPPORTED beyond).
 * Iteration histories, the frozen map, the
 * adjoint and smx_evaluate_static do not apply to it.
 */
int32_t smx_set_solver(smx_ctx ctx, int32_t solver);

/* One of SMX_FP64, SMX_BF16_3W, SMX_BF16_1W, SMX_FP32, SMX_FP16_2W. */
int32_t smx_set_precision(smx_ctx ctx, int32_t mode);

/*
 * Sign iteration of the FP64 path and of the reduced-precision bulk:
 * SMX_ITER_NS2 (default), X_{k+1} = X_k (3I - X_k^2) / 2, two products per
 * step (Sec. II-B); or SMX_ITER_PADE3, X_{k+1} = X_k (15I - 10X_k^2 +
 * 3X_k^4) / 8, the third-order Pade iteration of the paper's GPU runs (Sec.
 * VI-A), three products per step (T = X^2, W = (15I - 10T + 3T^2) / 8,
 * X W) with cubic convergence.  Same prescaling, stopping rules and
 * reduced-precision switch; the FP64 polish of the reduced-precision modes
 * stays Newton-Schulz.  Frozen evaluations, the mu search and the adjoint
 * follow the Newton-Schulz map only (SMX_E_UNSUPPORTED after a Pade
 * evaluation).
 */
int32_t smx_set_iteration(smx_ctx ctx, int32_t kind);

/*
 * Stopping rule of the iteration: stop at the first k with
 * max|X_k^2 - I| <= tol (FP64 products), at most max_iter steps.  In the
 * reduced-precision modes the bulk runs until tau_k = Tr(I - X_k^2) <=
 * switch_tol (tau_k bounds the largest 1 - x_i^2 over the eigenvalues x_i
 * of X_k, all of which lie in [-1, 1]), or until tau_k stops falling
 * (tau_k >= tau_{k-1}, or tau_k < 0.1 and tau_k > tau_{k-1}/2), or for at
 * most max_iter - n_polish
 * steps, and is followed by n_polish FP64 steps (1 <= n_polish <= 4 in these
 * modes), computed on the group's own columns only, since only those enter D:
 * X_{k+n_polish} E (E the own-column selector) is a polynomial of degree
 * 3^n_polish in the bulk result X_k, evaluated by 3^n_polish - 1 FP64 products
 * of X_k with n_g x m_own blocks.
 * Defaults: tol 1e-12, max_iter 100, n_polish 2, switch_tol 1e-3.
 */
int32_t smx_set_convergence(smx_ctx ctx, double tol, int32_t max_iter,
                            int32_t n_polish, double switch_tol);

/*
 * Step graphs.  With
 * steps_per_graph = S > 0 the Newton-Schulz step launches of each wave are
 * captured once into HIP graphs of S consecutive steps (all groups of the
 * wave, two product launches per step, three when frozen) and replayed;
 * groups that have converged skip on the device as before, and the host
 * polls the finished-group counter once per graph.  The graphs are kept
 * while the plan, buffers, precision and convergence settings stay the
 * same, and are captured again otherwise.  S = 0 (the default) launches
 * every product directly and records the per-launch profile
 * (smx_get_launch_profile reports no launches for graph replays).  Results
 * are bitwise the same either way.  SMX_E_INVALID unless 0 <= S <= 64.
 */
int32_t smx_set_graph(smx_ctx ctx, int32_t steps_per_graph);

/*
 * Launch order of the product tiles: 0 (default) deals each group's tiles to
 * one XCD (its L2), groups balanced over the 8 XCDs by work; 1 launches the
 * tiles group by group.  Takes effect at the next plan build.
 */
int32_t smx_set_tile_order(smx_ctx ctx, int32_t order);

/*
 * Operand stream of the reduced-precision word products: 0 (default) loads
 * each K step of both operand panels straight into LDS and waits for it;
 * 1 loads the next K step into registers while the matrix cores work on the
 * current one from LDS (groups with 3 n_pad^2 >= 2^31 words fall back to 0);
 * 2 launches the Newton-Schulz products of 2-word FP16 and 1-word BF16 on the
 * 128 x 128 bucket persistently: as many workgroups as the CUs hold, taking
 * tiles from one work list per XCD through atomic counters (each starts with
 * its own XCD's list, read from the hardware, then takes what the others left).
 * Results are bitwise the same.
 */
int32_t smx_set_kernel_variant(smx_ctx ctx, int32_t variant);

/*
 * Debug checks (0 off, the default; 1 on), for tracking down indexing errors:
 * smx_evaluate first validates every plan table on the host against the sizes
 * it indexes (slab, own-column and row-table offsets, block maps and offsets,
 * product tiles inside each group's lower triangle, gather chunks, scatter
 * blocks inside their submatrix; SMX_E_INVALID naming the table), and writes
 * a 64-KB guard pattern right after the extent the evaluation may write in
 * the arena, the polish pool and D (device memory the library owns); smx_wait
 * reads the guards back and returns SMX_E_HIP naming the buffer if a byte
 * changed.  Results are bitwise those without the checks.  Not applied to
 * smx_evaluate_static or to a caller work space (smx_set_workspace).
 */
int32_t smx_set_debug_checks(smx_ctx ctx, int32_t on);

/*
 * Size buckets of the 2-word FP16 and 1-word BF16 products (the paper
 * balances submatrices of uneven size over workers, Sec. IV-E; here the
 * uneven submatrices of one launch are split by size): groups whose padded
 * dimension n_pad is at least big_min_npad run on 256 x 256 output tiles
 * (one 512-lane workgroup per CU, operands double-buffered in LDS), the
 * others on 128 x 128 tiles; each bucket is one launch per product.
 * big_min_npad = 0 puts every group on 128 x 128 tiles.  Results are bitwise
 * the same for every choice.  Takes effect at the next plan build; other
 * precision modes always use 128 x 128 tiles.
 */
int32_t smx_set_tile_shape(smx_ctx ctx, int32_t big_min_npad);

/* The launch configuration in effect (outputs nullable): steps per graph
 * (smx_set_graph), tile launch order (smx_set_tile_order), size bucket
 * boundary (smx_set_tile_shape) and operand stream (smx_set_kernel_variant). */
int32_t smx_get_launch_config(smx_ctx ctx, int32_t *graph_steps, int32_t *tile_order,
                              int32_t *big_min_npad, int32_t *kernel_variant);

/*
 * Autotuner.  Times whole evaluations of the loaded problem (current
 * precision, groups and mu) for every candidate launch configuration, the
 * tile launch order (smx_set_tile_order) x steps per graph (0, 2, 8;
 * smx_set_graph) x, in the 2-word FP16 and 1-word BF16 modes, the size bucket
 * boundary of the 256 x 256 tiles (0, 384, 640, 896; smx_set_tile_shape): one
 * untimed run per candidate, then the minimum device time of `reps` runs.  It
 * applies the fastest and returns it (outputs nullable; the bucket boundary
 * through smx_get_launch_config).  If the environment variable SMX_TUNE_CACHE
 * names a file, the choice is appended there as "key graph_steps tile_order
 * big_min_npad ms", keyed by device architecture, precision and the batch
 * shape.  With use_cache != 0 a matching record is applied without timing.
 * Invalidates results.
 */
int32_t smx_autotune(smx_ctx ctx, int32_t reps, int32_t use_cache, int32_t *graph_steps_out,
                     int32_t *tile_order_out, double *best_ms_out);

/*
 * Device work space.  The dense submatrices are processed in waves of
 * consecutive groups; all groups of a wave are resident together (three FP64
 * n_pad x n_pad slabs per group, the reduced-precision words laid over
 * two of them, 26 bytes per element, plus 72 n_pad m_own bytes of own-column
 * blocks), and the waves reuse one arena.  bytes = 0 (the default) sizes the
 * waves to the free device memory at plan time, less the plan's tables and
 * 1 GiB, and at most 3/4 of the device; bytes > 0 caps the arena and forces
 * more waves.  A group that does
 * not fit alone fails with SMX_E_NOMEM.  Results do not depend on the wave
 * split (bitwise).  With more than one wave, smx_backward is unsupported and
 * smx_get_submatrix(what = 1) serves only the last wave's groups.  Takes
 * effect at the next call that builds the plan; invalidates results.
 */
int32_t smx_set_workspace_limit(smx_ctx ctx, int64_t bytes);

/*
 * Caller-owned work space, e.g. a torch tensor.  smx_workspace_size gives the
 * bytes of a work space that holds every submatrix of the loaded problem at
 * once (one wave): the arena of dense slabs / reduced-precision words (26
 * bytes per padded element) and the own-column blocks of the polish (72
 * bytes per n_pad x m_own element), with alignment slack.  It builds the plan
 * for the current groups if needed.
 * smx_set_workspace(ctx, dptr, bytes) makes evaluations use [dptr, dptr +
 * bytes) instead of memory the library allocates: dptr is device memory of
 * the context's device, 256-byte aligned; the caller keeps it allocated and
 * does not touch it while the context may use it (until the next
 * smx_set_workspace or smx_destroy).  A work space smaller than
 * smx_workspace_size runs the groups in waves (as smx_set_workspace_limit);
 * one too small for the largest group makes evaluations fail with
 * SMX_E_NOMEM.  dptr = NULL with bytes = 0 returns to library-allocated
 * memory.  Results are bitwise those of the library-allocated arena.  The
 * adjoint (smx_backward) and the mu tangent of frozen evaluations keep using
 * library-allocated buffers.  Synchronises the stream; invalidates results.
 */
int32_t smx_workspace_size(smx_ctx ctx, size_t *bytes);
int32_t smx_set_workspace(smx_ctx ctx, void *dptr, size_t bytes);

/*
 * Host polling.  on = 1 (default): smx_evaluate reads the finished-group
 * counter one step (or one step graph) behind the device and stops enqueueing
 * steps once every group is done, which synchronises the host with the stream
 * during the call.  on = 0: smx_evaluate enqueues every step up to the cap
 * (max_iter, or max_iter - n_polish bulk steps) without waiting on the
 * device; finished groups skip on the device, so results are bitwise the
 * same, at the cost of the launches past convergence.  With smx_set_graph the
 * steps are replayed from graphs either way.
 */
int32_t smx_set_host_poll(smx_ctx ctx, int32_t on);

/*
 * Evaluate D, N and E for the current K, groups and mu.  The work is
 * enqueued on the context's stream; the call returns after enqueueing it
 * (with host polling on, the host only polls a small counter to stop the
 * iteration when every group has converged).  D stays resident on the device.
 */
int32_t smx_evaluate(smx_ctx ctx);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as smx_evaluate, with every piece of work memory (the plan's
 * tables, the iteration state, the dense submatrices or their words, the
 * polish blocks) taken from one fixed device array of
 * SMX_STATIC_SCRATCH_BYTES inside the library (one per device, held until the
 * process ends).  The call allocates nothing: no device or pinned memory, no
 * events, no graphs.  K and D are the context's (allocated by smx_load_k).
 * Groups run in waves sized to the array; a problem whose tables, state and
 * largest group do not fit returns SMX_E_NOMEM before anything is enqueued.
 * All steps up to the cap are enqueued without host polling (as with
 * smx_set_host_poll(0)); finished groups skip on the device.  Results (D, N,
 * E, the status of smx_wait) are bitwise those of smx_evaluate.  Per-group
 * details are not kept: smx_get_stats, smx_get_group_info, smx_get_history,
 * smx_get_launch_profile, smx_get_submatrix(what = 1), smx_set_frozen and
 * smx_backward return SMX_E_STATE after it.  Frozen evaluations are refused
 * (SMX_E_UNSUPPORTED).  Every static evaluation on a device shares that
 * device's array: calls that overlap in time on one device (other threads,
 * other streams) race and give undefined results.
 */
#define SMX_STATIC_SCRATCH_BYTES (1024ull * 1024ull * 1024ull)
int32_t smx_evaluate_static(smx_ctx ctx);

/*
 * D of the last evaluation written into another layout of n_out stored
 * values: out[index[q]] = D_q for every stored value q of the loaded problem
 * and 0 at every other position (the split problem of smx_split_columns back
 * in K's layout, index = its e_src: elements the split dropped get D = 0).
 * index: host, nvalues entries, each in [0, n_out) and pairwise distinct
 * (SMX_E_INVALID otherwise).  out: host, or device when out_on_device != 0.
 * Synchronises.
 */
int32_t smx_get_d_expanded(smx_ctx ctx, const int64_t *index, int64_t n_out, double *out,
                           int32_t out_on_device);

/* Wait for the last evaluation.  SMX_E_NONFINITE if an iterate was not
 * finite; SMX_E_NOT_CONVERGED (D is still written) if any group did not
 * converge:
 *   SMX_FP64: max|X_k^2 - I| > tol at k = max_iter;
 *   reduced-precision modes: the bulk left above switch_tol (stall rule or
 *   step cap; for SMX_BF16_1W, whose rounding floor lies above switch_tol by
 *   design, above 0.1), or the own-column residual r = max|X_{k+p-1}^2 E - E|
 *   of the polish gives 3 r^2 / 4 > tol, i.e. the returned iterate misses the
 *   FP64 stopping rule.  Convergence is about the iteration, not accuracy:
 *   SMX_BF16_1W converges to the sign of its rounded iterate (~1e-3 off). */
int32_t smx_wait(smx_ctx ctx);

/* Copy D (K's layout, same number of doubles as K's values) into `out`
 * (host, or device when out_on_device != 0).  Synchronises. */
int32_t smx_get_d(smx_ctx ctx, double *out, int32_t out_on_device);

/* N = Tr D and E = Tr(D K) of the last evaluation, FP64, reduced in a fixed
 * order (bitwise reproducible).  Synchronise. */
int32_t smx_trace(smx_ctx ctx, double *n_out);
int32_t smx_energy(smx_ctx ctx, double *e_out);

/* Summary of the last evaluation.  Synchronises. */
int32_t smx_get_stats(smx_ctx ctx, smx_stats *out);

/*
 * Per-group details of the last evaluation (host arrays of ngroups entries,
 * any may be NULL): submatrix dimension n_g, iterations k_g, Gershgorin
 * scale s_g, and the last computed max|X^2 - I|.  Synchronises.
 */
int32_t smx_get_group_info(smx_ctx ctx, int32_t *n_g, int32_t *iters,
                           double *scale, double *resid);

/*
 * Convergence history of the last evaluation (the involutority and trace
 * histories behind the paper's GPU convergence plot, Sec. VI-A): for every
 * group g, nsteps[g] = k_g + 1 bulk steps were taken (k_g: the step whose
 * X_k was the bulk result), and for k < min(cap, nsteps[g]):
 *   resid[g * cap + k] = max|X_k^2 - I| (FP64 mode: over the true n_g x n_g
 *       block in FP64; reduced-precision modes: over its lower triangle, from
 *       the FP32-accumulated square),
 *   tau[g * cap + k]   = Tr(I - X_k^2) (reduced-precision modes; NaN in FP64
 *       mode, which does not form it).
 * Entries k >= nsteps[g] are NaN.  Host arrays of ngroups * cap (resid, tau)
 * and ngroups (nsteps) entries, each nullable.  Synchronises.
 */
int32_t smx_get_history(smx_ctx ctx, int32_t cap, double *resid, double *tau, int32_t *nsteps);

/*
 * Dense submatrix of group g (Sec. III-A: the submatrix a_i and its result
 * f(a_i)), column-major n_g x n_g into host array `out` with leading
 * dimension ld >= n_g:
 *   what = 0: A_g = K[R(g), R(g)] - mu I as gathered on the device
 *             (needs a loaded K; uses the current groups and mu);
 *   what = 1: the sign S_g of the last evaluation (the whole submatrix,
 *             not only the group's own columns); in the reduced-precision
 *             modes the bulk's last iterate in FP64, before the polish
 *             (which is computed on the own columns only).
 * n_out (nullable) receives n_g.  With out == NULL only n_g is returned.
 * Synchronises.  what = 0 overwrites scratch that what = 1 does not read.
 */
int32_t smx_get_submatrix(smx_ctx ctx, int32_t g, int32_t what, double *out, int32_t ld,
                          int32_t *n_out);

/*
 * Frozen iteration.  With on != 0 (after an evaluation), later evaluations
 * take exactly the step counts k_g of that evaluation (FP64 steps, polish
 * included) and its scales s_g, instead of the stopping rule and a fresh
 * Gershgorin bound: the map K, mu -> D is then a fixed polynomial, which is
 * what derivatives and the mu search act on.  Frozen evaluations run in
 * SMX_FP64 only and also carry the mu tangent of the iteration (one more
 * symmetric product per step) for smx_dn_dmu.  on = 0 unfreezes.
 */
int32_t smx_set_frozen(smx_ctx ctx, int32_t on);

/* dN/dmu of the last (frozen) evaluation: -1/2 times the own-diagonal trace of
 * the tangent dX_k/dmu, with dX_0/dmu = -I/s_g.  Synchronises. */
int32_t smx_dn_dmu(smx_ctx ctx, double *out);

/*
 * Chemical potential for a target electron count (Sec. IV-G, Algorithm 1
 * reads n_elec off fixed decompositions; here the iteration itself is
 * frozen).  Bracket: the Gershgorin interval of K; scales s_g: the larger of
 * the bracket ends' ||K_sub - mu I||_inf (valid for every mu inside); step
 * counts: one converged FP64 evaluation at the current mu with those scales.
 * Then safeguarded Newton on the frozen N(mu) with dN/dmu from the tangent,
 * until |N - n_target| <= tol or max_steps evaluations.  Leaves the context
 * at mu_out (unfrozen); *steps_out (nullable) = evaluations used.  Returns
 * SMX_E_NOT_CONVERGED if the tolerance was not reached.
 */
int32_t smx_find_mu(smx_ctx ctx, double n_target, double tol, int32_t max_steps,
                    double *mu_out, int32_t *steps_out);

/*
 * Chemical potential by the paper's Algorithm 1 (Sec. IV-G): every submatrix
 * is diagonalised once at the current mu (as SMX_SOLVER_EIG, at the current
 * kT), which gives its eigenvalues lambda_gl and weights w_gl = sum over the
 * own columns c of Q_cl^2; then N(mu) = sum_g sum_l w_gl f(lambda_gl - mu)
 * (monotone in mu) is bisected without solving again, 128 trial values per
 * step inside the bracket of K's Gershgorin interval (widened by 40 kT),
 * until |N - n_target| <= tol or max_steps steps.  D, N and E are then formed
 * at mu_out from the stored decompositions (with more than one wave, by a new
 * evaluation at mu_out), and the context is left at mu_out.  *steps_out
 * (nullable) = bisection steps.  At kT = 0 N(mu) is a staircase and may step
 * over n_target: SMX_E_NOT_CONVERGED (mu_out at the step, D still formed).
 */
int32_t smx_find_mu_eig(smx_ctx ctx, double n_target, double tol, int32_t max_steps,
                        double *mu_out, int32_t *steps_out);

/*
 * Spectrum of the last diagonalisation (smx_evaluate with SMX_SOLVER_EIG or
 * kT > 0, or smx_find_mu_eig): for every group g in order, its n_g
 * eigenvalues of K[R(g), R(g)] (no shift; ascending within each unreduced
 * block of the tridiagonal form) and Algorithm 1's weights w_gl.  Host arrays
 * of sum_g n_g entries, each nullable.  Synchronises.
 */
int32_t smx_get_spectrum(smx_ctx ctx, double *lam, double *w);

/*
 * Reverse-mode derivative of L = gE E + gN N + <gD, D> (gD nullable, K's
 * layout, host or device) through the frozen map of the last evaluation:
 * its step counts k_g and scales s_g are held fixed, and the iterates are
 * recomputed in FP64 from checkpoints kept every 8 steps.  Per step the
 * adjoint is Xb_k = (3 Xb - Xb X_k^2 - X_k^2 Xb - X_k Xb X_k) / 2 (the
 * transpose of the derivative of X (3I - X^2) / 2), seeded at the sign with
 * the symmetrised -1/2 dL/dD of the own columns; A_g = K_sub - mu I and
 * X_0 = A_g / s_g give dK by the transpose of the gather, plus gE D for the
 * explicit K in E = Tr(DK).
 *   dK_out (nullable; host, or device when dK_on_device != 0): dL/dK for
 *   every stored value of K, each treated as an independent variable; since
 *   only symmetric changes of K are meaningful, the symmetric part
 *   dK_IJ + dK_JI^T is what is fixed (each group's part is symmetrised).
 *   dmu_out (nullable): dL/dmu = -sum_g tr(dL/dA_g).
 * Needs free device memory for 4 + 8 + k_max/8 + 1 work slabs.  Synchronises.
 */
int32_t smx_backward(smx_ctx ctx, double gE, double gN, const double *gD, int32_t gD_on_device,
                     double *dK_out, int32_t dK_on_device, double *dmu_out);

/*
 * Group selection (Sec. IV-C, "Generating Submatrices From Multiple Block
 * Columns").  Context-free host functions on a block pattern (the layout of
 * smx_load_k, values not needed); errors are described by
 * smx_group_last_error().
 *
 * smx_group_speedup: the estimated additional speedup of Eq.
 * estimatedspeedup, S = sum over the single block columns j of n_j^3 divided
 * by sum over the given groups g of n_g^3, n the dimension of the submatrix
 * (the sizes of the union of the stored block rows of the columns); the
 * evaluation of each submatrix is taken to cost O(n^3).  *work_out
 * (nullable) = sum_g n_g^3.
 */
int32_t smx_group_speedup(int32_t nblk, const int32_t *blk_size, const int64_t *col_ptr,
                          const int32_t *row_idx, int32_t ngroups, const int32_t *grp_ptr,
                          const int32_t *grp_blocks, double *s_out, double *work_out);

/*
 * smx_group_kmeans: block columns that sit close together in space are
 * combined (the paper clusters the atoms' positions with k-means, one
 * position per block column).  coords: nblk x 3 (row-major) positions; box
 * > 0: cubic periodic box of that edge (minimum-image distances, circular
 * means), box = 0: plain Euclidean space.  k-means++ seeding from `seed`
 * (deterministic), at most max_iter Lloyd iterations (nearest centre, lowest
 * index on ties).  Output: *ngroups_out <= nclusters non-empty groups in the
 * order of their first block column, block columns ascending inside each, as
 * grp_ptr_out (nclusters + 1 entries of room) and grp_blocks_out (nblk),
 * ready for smx_set_groups.
 */
int32_t smx_group_kmeans(int32_t nblk, const double *coords, double box, int32_t nclusters,
                         int32_t seed, int32_t max_iter, int32_t *ngroups_out,
                         int32_t *grp_ptr_out, int32_t *grp_blocks_out);

/*
 * Splitting submatrices (Sec. IV-C, "Splitting up submatrices"): a dense
 * submatrix may still be sparse element by element, and applying the
 * submatrix method to it a second time, for the columns it owns only, gives
 * one smaller sub-submatrix per column.  The sub-submatrix of column c keeps
 * the rows r with r = c or |K_rc| > eps (r in a stored block of c's block
 * column); it does not depend on the group of c's block column, so the whole
 * split problem is the submatrix method on K at the level of single elements.
 * This call builds that problem, ready for smx_load_k / smx_set_groups:
 * n (the sum of the block sizes) columns, each a block of size 1; e_col_ptr (n + 1),
 * e_row_idx and e_values (nnz, rows ascending per column) the kept elements;
 * e_src (nnz) the position of each kept element in `values`; groups
 * e_grp_ptr (ngroups + 1) / e_grp_cols (n): single columns, or with merge != 0
 * runs of consecutive columns of one block column that keep the same rows
 * (one sub-submatrix serves them all; the result is the same).  Call once
 * with e_col_ptr = NULL for *n_out, *nnz_out and *ngroups_out, then with
 * arrays of those sizes.  values: host, K's layout (smx_load_k).  D of the
 * split problem goes back to K's layout with smx_get_d_expanded(e_src).
 * Errors as the group-selection calls (smx_group_last_error).
 */
int32_t smx_split_columns(int32_t nblk, const int32_t *blk_size, const int64_t *col_ptr,
                          const int32_t *row_idx, const double *values, double eps, int32_t merge,
                          int32_t *n_out, int64_t *nnz_out, int32_t *ngroups_out, int64_t *e_col_ptr,
                          int32_t *e_row_idx, double *e_values, int64_t *e_src, int32_t *e_grp_ptr,
                          int32_t *e_grp_cols);

/* Message for the last failing group-selection call (never NULL). */
const char *smx_group_last_error(void);

/* Number of groups and stored values of the loaded problem. */
int32_t smx_get_sizes(smx_ctx ctx, int32_t *ngroups, int64_t *nvalues);

/*
 * Per-launch profile of the matrix-core product kernels of the last
 * evaluation, in launch order: device time in ms measured with HIP events on
 * the context's stream, the algorithmic flops of the launch (2 n_g^3 for
 * every group the launch works on, i.e. one dense n_g x n_g product), and
 * its kind: 0/1 FP64 square/update, 2/3 reduced-precision square/update on
 * 128 x 128 tiles, 4/5 FP64 polish square/update, 6 mu tangent, 7/8
 * reduced-precision square/update on 256 x 256 tiles, 9/10 reduced-precision
 * Pade combine on 128 x 128 / 256 x 256 tiles, 11 FP64 Pade combine (the Pade
 * square shares the square's kind), 12 Householder reduction of the
 * diagonalisation path (algo_flops 4/3 n_g^3 per group).  Writes min(cap, count) entries to the host
 * arrays (any may be NULL) and the launch count to *count.  Synchronises.
 */
int32_t smx_get_launch_profile(smx_ctx ctx, int32_t cap, float *ms, double *algo_flops,
                               int32_t *kind, int32_t *count);

/*
 * Issued matrix-core flops of each launch of smx_get_launch_profile, in the
 * same order: 2 x 64 x 64 x n_pad per live 64 x 64 wave tile of a 128 x 128
 * tile (2 x 16 x 16 x n_pad per live 16 x 16 block of a 256 x 256 tile),
 * times the word products per algorithmic product (3 for SMX_FP16_2W, 6 for
 * SMX_BF16_3W, else 1), padding included, for every group the launch works
 * on; kind 12 (vector units only) repeats its algorithmic flops.  Divided by
 * the launch time and the matrix-core peak of the format this is the
 * fraction of the matrix cores the launch kept busy.  Writes min(cap, count)
 * entries (issued_flops may be NULL) and the launch count to *count.
 * Synchronises.
 */
int32_t smx_get_launch_issued(smx_ctx ctx, int32_t cap, double *issued_flops, int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* SMX_H */
