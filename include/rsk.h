/*
 * rsk.h -- C ABI of librsk, the gfx950 implementation of the averaged
 * randomized sparse Kaczmarz method (RSKA) of Tondji & Lorenz,
 * "Faster Randomized Block Sparse Kaczmarz by Averaging".
 *
 * The method (eq. (rska) and Algorithm 1 of the paper) solves
 *     min_x  lambda ||x||_1 + 1/2 ||x||^2   s.t.  A x = b
 * by iterating, from x*_0 = x_0 = 0,
 *     x*_{k+1} = x*_k - (alpha_k/eta) sum_{t<eta} (<a_{tau_t}, x_k> - b_{tau_t}) / ||a_{tau_t}||^2 * a_{tau_t}
 *     x_{k+1}  = S_lambda(x*_{k+1}),   S_lambda(v) = max(|v| - lambda, 0) sign(v)
 * where tau_k = (tau_0..tau_{eta-1}) are eta row indices drawn with
 * replacement (uniform weights w_i = alpha, variant v2 of Sec. 5).
 *
 * Conventions shared by every entry point:
 *  - Every array pointer is a DEVICE pointer owned by the caller. The library
 *    never allocates, frees or retains them past the call; buffers must stay
 *    alive until the work queued on `stream` has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on that stream.
 *  - Host-side validation happens before anything is queued; on failure the
 *    call returns RSK_ERR_INVALID_ARG / RSK_ERR_UNSUPPORTED / RSK_ERR_WORKSPACE
 *    and queues nothing.
 *  - Faults found on the device (an index >= m in the stream, a referenced row
 *    with ||a_i|| = 0, a non-finite coefficient) are written to
 *    status_dev[0] (first error wins) and end the launch at the step where
 *    they occur, for every workgroup alike. status_dev[1] receives the number
 *    of completed steps. The caller reads status_dev after synchronising.
 *  - Dense matrices are row-major with leading dimension ld >= n (elements).
 *    dtype RSK_F32 or RSK_F64; b, x*, x, rownorm2, alpha_k and y use the
 *    same dtype as A.
 *  - The index stream is int32, step-major: step k uses
 *    index_stream[stream_offset + k*eta + t], t = 0..eta-1.
 *  - Workspace: query its size with the matching rsk_workspace_size_* call;
 *    the solve uses it for cross-workgroup exchange and scratch, and it must
 *    be 256-byte aligned.
 */
#ifndef RSK_H
#define RSK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSK_ABI_VERSION 6

typedef enum { RSK_F32 = 0, RSK_F64 = 1 } rsk_dtype;

typedef enum {
  RSK_OK = 0,
  RSK_ERR_INVALID_ARG = 1, /* null pointer, bad size, eta < 1, K < 0, lambda < 0, alpha <= 0 or not finite */
  RSK_ERR_UNSUPPORTED = 2, /* dtype, alignment or size the kernels do not take */
  RSK_ERR_WORKSPACE = 3,   /* workspace too small or misaligned */
  RSK_ERR_HIP = 4,         /* a HIP runtime call failed (launch, occupancy query) */
  RSK_ERR_ZERO_ROW = 5,    /* device: the stream references a row with ||a_i|| = 0 (Algorithm 1 requires a_i != 0) */
  RSK_ERR_INDEX_RANGE = 6, /* device: a stream index (or CSR column) outside its range */
  RSK_ERR_NONFINITE = 7,   /* device: a coefficient became inf/nan (alpha beyond the stability bound of Theorem 1) */
  RSK_ERR_ABORTED = 8      /* device: a bounded wait inside the persistent kernel expired */
} rsk_status;

/* Dense row-major matrix: element (i,j) at val[i*ld + j]. */
typedef struct {
  int64_t m, n, ld;
  int32_t dtype;
  const void *val;
} rsk_dense;

/* CSR matrix: row i holds col[row_ptr[i] .. row_ptr[i+1]) and the matching val. Columns in [0,n). */
typedef struct {
  int64_t m, n, nnz;
  int32_t dtype;
  const int64_t *row_ptr;
  const int32_t *col;
  const void *val;
} rsk_csr;

/* Parameters of one solve (Algorithm 1's Require line plus run control). */
typedef struct {
  double lambda;               /* >= 0; lambda = 0 is the (relaxed) randomized Kaczmarz special case */
  int32_t eta;                 /* >= 1 rows per step */
  double alpha;                /* > 0 uniform relaxation w_i = alpha; used when alpha_k == NULL */
  const void *alpha_k;         /* nullable device array of K per-step relaxations (dtype of A) */
  int64_t K;                   /* >= 0 steps */
  const int32_t *index_stream; /* device, >= stream_offset + K*eta entries */
  int64_t stream_offset;       /* >= 0 */
  const void *rownorm2;        /* device, m entries ||a_i||^2 (from rsk_rownorm2_*), dtype of A */
  int32_t warm_start;          /* 0: x*_0 = 0 (the paper); 1: start from the x_star passed in */
  const void *x_ref;           /* nullable device vector (n): monitor target */
  int64_t check_every;         /* > 0 with x_ref: every check_every steps record ||x - x_ref||/||x_ref|| */
  double tol;                  /* with the monitor: stop early once the relative error is <= tol (0 = never) */
  double *err_hist;            /* nullable device array, K/check_every entries (double) */
  void *y_out;                 /* nullable device array (m, dtype of A), in/out: y[tau_t] -= c_t, so x* = A^T y.
                                  CSR and dense kernel 4: each row's slots of a step are applied once, in a
                                  fixed order, so y is bitwise reproducible. Dense kernels 1-3: summed with
                                  floating-point atomics, so where a row is drawn more than once in a step y
                                  is reproducible to rounding only (x* and x stay bitwise reproducible) */
  int32_t *status_dev;         /* device int32[2]: [0] status (0 = ok), [1] steps completed. Required. */
  int32_t grid;                /* workgroups of the persistent kernel; 0 = chosen by the library */
  int32_t kernel;              /* dense kernel: 0 = chosen by the library, 1 = general, 2 = float32 register
                                  tile, 3 = float32 register tile over two row groups, 4 = one workgroup
                                  with the step in registers (see rsk_avg_solve_dense); CSR: 0, 1 or 2;
                                  multi-RHS: 0..3 (see rsk_avg_solve_multirhs) */
  const void *row_w;           /* nullable device array (m, dtype of A): per-row weights w_i, the diagonal W of
                                  Definition 1 (variants v3/v4 of Sec. 5); row i is relaxed by alpha (or
                                  alpha_k[k]) times w_i. Dense, CSR and multi-RHS solves; not the adjoint or
                                  the block method. */
} rsk_params;

/*
 * One system of a batch (rsk_avg_solve_batched). All pointers inside are
 * device pointers. The solve takes the array twice: in host memory (checked
 * and planned on the host) and the same bytes in device memory (read by the
 * kernels).
 */
typedef struct {
  const void *A;               /* row-major m x n, leading dimension ld, dtype of the batch */
  int64_t m, n, ld;
  const void *b;               /* m */
  const void *rownorm2;        /* m, ||a_i||^2 */
  const int32_t *index_stream; /* K*eta entries, step-major, this system's own stream */
  int64_t K;                   /* steps (upper bound when a tolerance stops the system early) */
  int32_t eta;                 /* rows per step, >= 1 */
  int32_t warm_start;          /* 1: start from x_star */
  double alpha, lambda;
  void *x_star;                /* n, in/out */
  void *x;                     /* n, out */
  const void *x_ref;           /* nullable monitor target (n) */
  int64_t check_every;         /* monitor period, with x_ref */
  double tol;                  /* stop this system once ||x - x_ref||/||x_ref|| <= tol (0: never) */
  double *err_hist;            /* nullable, K/check_every entries */
  int32_t *status_dev;         /* int32[2]: status, steps completed */
} rsk_batch_item;

/*
 * Row sampler (the index stream of Sec. 1.1 generated on the device).
 *
 * rsk_sampling_cdf_dense: cdf_i = sum_{j <= i} ||a_j||^2 in double (device,
 * m entries), row norms accumulated in double, running sums by a three-pass
 * scan (chunk sums, a fixed-order scan of the chunk sums, chunk-local scans):
 * equal to a sequential running sum up to rounding order, the same bits on
 * every run. Workspace: rsk_workspace_size_sampling_cdf(m).
 *
 * rsk_sample_stream: out[(k - k0) * eta + t] for k0 <= k < k0 + K, t < eta
 * (device int32, step-major, the layout every solve takes as index_stream):
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) of the counter
 * (t, k mod 2^32, k div 2^32, 0) under the key (seed mod 2^32, seed div 2^32)
 * gives words w0, w1; u = ((w0 >> 5) 2^26 + (w1 >> 6)) / 2^53 in [0, 1); the
 * index is the first i with cdf[i] > u * cdf[m-1] (at most m-1), i.e. rows
 * are drawn with replacement with P(i) = ||a_i||^2 / ||A||_F^2. The result is
 * a function of (cdf, seed, k, t) only. cdf must be non-decreasing with a
 * positive finite last entry (otherwise every index is m-1). m <= 2^31 - 1.
 */
int32_t rsk_workspace_size_sampling_cdf(int64_t m, size_t *bytes);
int32_t rsk_sampling_cdf_dense(const rsk_dense *A, double *cdf, void *workspace, size_t ws_bytes, void *stream);
/* The same running sums of ||a_i||^2 / w_i (row_w: device, m, dtype of A): the probabilities
 * p_i proportional to ||a_i||^2 / w_i of variant v4 (Sec. 5), coupled to the per-row weights of
 * rsk_params.row_w as in Assumption 1. Same workspace. */
int32_t rsk_sampling_cdf_dense_weighted(const rsk_dense *A, const void *row_w, double *cdf, void *workspace,
                                        size_t ws_bytes, void *stream);
/* Running sums of arbitrary non-negative weights (device double, m): cdf for any sampling
 * distribution p_i proportional to weights[i]. Same scan and workspace size. */
int32_t rsk_sampling_cdf_weights(const double *weights, int64_t m, double *cdf, void *workspace, size_t ws_bytes,
                                 void *stream);
int32_t rsk_sample_stream(const double *cdf, int64_t m, uint64_t seed, int64_t k0, int64_t K, int32_t eta,
                          int32_t *out, void *stream);

/*
 * Linearized Bregman method: the full-batch comparator of Sec. 4 (the block
 * step of eq. (bsk) with every row in the block and the step 1/||A||_2^2 of
 * the remark on its linear rate; the paper cites Cai, Osher and Shen and Yin
 * for it). From x*_0 = 0, x_0 = 0 (or the x* passed in, with x_0 = S_lambda(x*_0)):
 *   x*_{k+1} = x*_k - step A^T (A x_k - b),   x_{k+1} = S_lambda(x*_{k+1}).
 * One iteration reads A once (a row-blocked pass forming A x_k - b and
 * A^T (A x_k - b) together) and n-sized vectors a few times. All sums are in
 * fixed orders: the results are the same bits on every run.
 *
 * rsk_workspace_size_lb_dense: device workspace bytes for A (256-byte aligned).
 * rsk_lb_solve_dense: A device row-major (rsk_dense), b device (m), x_star and
 *   x device (n, dtype of A): x_star in (warm_start) and out, x out. Fails with
 *   RSK_ERR_UNSUPPORTED for n > 6144 * (16 / sizeof element) (n > 6144 when A
 *   is not 16-byte aligned or ld is not a multiple of 16 / sizeof element).
 *   Device status as in rsk_params (RSK_ERR_NONFINITE when x* leaves the
 *   finite range; status_dev[1] = iterations run).
 * rsk_spectral_norm2_dense: sigma_max(A)^2 by `iters` >= 1 steps of power
 *   iteration on A^T A from v_j = 1 + (j mod 7)/7 (normalised): w = A^T A v,
 *   est = <v, w>, v = w / ||w||. est: device double; v: device (n, dtype of
 *   A), out: the last unit vector. Same workspace as rsk_lb_solve_dense.
 */
typedef struct {
  double lambda;       /* >= 0 */
  double step;         /* > 0; the paper's choice is 1 / sigma_max(A)^2 (rsk_spectral_norm2_dense) */
  int64_t K;           /* >= 0 iterations */
  int32_t warm_start;  /* 1: start from the x_star passed in */
  const void *x_ref;   /* nullable device vector (n): monitor target */
  int64_t check_every; /* > 0 with x_ref: every check_every iterations record ||x - x_ref||/||x_ref|| */
  double *err_hist;    /* nullable device array, K/check_every entries */
  double *res_hist;    /* nullable device array, K entries: ||A x_k - b|| of the iterate step k starts from */
  int32_t *status_dev; /* device int32[2]: [0] status, [1] iterations run. Required. */
} rsk_lb_params;

int32_t rsk_workspace_size_lb_dense(const rsk_dense *A, size_t *bytes);
int32_t rsk_lb_solve_dense(const rsk_dense *A, const void *b, const rsk_lb_params *p, void *x_star, void *x,
                           void *workspace, size_t ws_bytes, void *stream);
int32_t rsk_spectral_norm2_dense(const rsk_dense *A, int64_t iters, void *v, double *est, void *workspace,
                                 size_t ws_bytes, void *stream);

/*
 * Block sparse Kaczmarz, eq. (bsk) (Sec. 1.1): per step the eta rows tau_k of
 * the index stream form A_tau (a repeated index is a repeated row) and
 *   x*_{k+1} = x*_k - w A_tau^T (A_tau x_k - b_tau) / ||A_tau||_2^2,
 *   x_{k+1} = S_lambda(x*_{k+1}),
 * with w = p->alpha. ||A_tau||_2^2 is the largest eigenvalue of the block's
 * Gram matrix A_tau A_tau^T, computed in double to rounding (Householder
 * tridiagonalisation, then Sturm-count bisection) for every step before the
 * iteration starts (it does not depend on x); the iteration is the RSKA solve
 * with unit row norms and per-step relaxation alpha_k = eta w / ||A_tau_k||^2.
 * Takes the rsk_params of rsk_avg_solve_dense with 1 <= eta <= 64, alpha = w,
 * alpha_k null; rownorm2 is ignored; y_out, the monitor, tol, grid and kernel
 * mean what they mean there. block_norm2: nullable device double[K],
 * ||A_tau_k||_2^2 of every step. Device status: RSK_ERR_INDEX_RANGE (stream
 * index outside [0, m)), RSK_ERR_ZERO_ROW (a block of zero rows: that step
 * leaves x* unchanged), RSK_ERR_NONFINITE. x* and x are bitwise reproducible
 * (y_out: see rsk_params).
 */
int32_t rsk_workspace_size_bsk_dense(const rsk_dense *A, const rsk_params *p, size_t *bytes);
int32_t rsk_bsk_solve_dense(const rsk_dense *A, const void *b, const rsk_params *p, void *x_star, void *x,
                            double *block_norm2, void *workspace, size_t ws_bytes, void *stream);

/*
 * Tuning table. The choices a solve makes when the caller leaves them to the
 * library (rsk_avg_solve_dense with kernel = 0 and grid = 0, the two product
 * splits of rsk_avg_solve_multirhs and rsk_avg_adjoint, the per-system
 * workgroup targets of rsk_avg_solve_batched with wg_bytes = 0) are read from
 * a process-global table that a tuner fills with measured winners; where the
 * table has no entry, the built-in rules apply. The table only selects among
 * launches the library supports: results are those of the explicit choice,
 * bit for bit, and a tuned choice that does not apply to a matrix (alignment,
 * leading dimension) falls back to the built-in rule.
 *   path RSK_TUNE_DENSE:    key (dtype, m, n, eta);    v0 = kernel (1..4), v1 = grid.
 *   path RSK_TUNE_MULTIRHS: key (dtype, m, n, eta, R); v0 = S (splits of the n columns in
 *                           A_tau X), v1 = S2 (row splits of A_tau^T C: 1, 2, 4 or 8), v2 = the
 *                           kernel (1 step kernels, 2 one persistent launch, 3 wide-tile step
 *                           kernels; 0 = built-in). The adjoint takes the tile of v2 = 3 as well.
 *   path RSK_TUNE_BATCHED:  key (dtype, m = the class's upper bound on a system's step bytes
 *                           eta * n * element size; n = eta = 0; R = the batched launch: 0
 *                           general kernel, 2 register tile); v0 = row bytes per workgroup for
 *                           systems of that class in that launch (a system takes the class
 *                           with the smallest bound >= its step bytes; at most 8 classes).
 * `us` is the measured time of the choice (informational). The cache file
 * (rsk_tune_save / rsk_tune_load) is text, one entry per line:
 * "path dtype m n eta R v0 v1 v2 us". If the environment variable RSK_TUNE_CACHE
 * names a file, it is loaded at the first lookup. All calls are thread-safe;
 * a table changed between a workspace query and its solve can make the solve
 * return RSK_ERR_WORKSPACE.
 */
enum { RSK_TUNE_DENSE = 0, RSK_TUNE_MULTIRHS = 1, RSK_TUNE_BATCHED = 2 };
typedef struct {
  int32_t path, dtype;
  int64_t m, n;
  int32_t eta, R;
  int64_t v0, v1, v2;
  double us;
} rsk_tune_entry;
int32_t rsk_tune_set(const rsk_tune_entry *e);                                   /* install or replace */
int32_t rsk_tune_get(const rsk_tune_entry *key, rsk_tune_entry *out, int32_t *found);
int32_t rsk_tune_erase(const rsk_tune_entry *key);                               /* one key, if present */
int32_t rsk_tune_clear(int32_t path);                                            /* path < 0: every entry */
int32_t rsk_tune_load(const char *path);                                         /* merge a cache file */
int32_t rsk_tune_save(const char *path);

/*
 * Measurement, not a solve: the HBM reads of a float32 register-tile solve on
 * `grid` workgroups in `row_groups` row groups (1, 2, 4 or 8), alone. For K
 * steps, workgroup g reads the part of step k's sampled rows (index_stream,
 * step-major, K * eta entries) that it would hold in such a solve: its row
 * group's rows of the step and its column slice (whole 16-float units, the
 * solve's XCD-aware slice order), with no exchange and no update. The time of
 * the call against K * eta * n * 4 bytes is the rate HBM serves that pattern
 * of row pieces at, the ceiling of the solve's own rate (eq. (rska) reads
 * each sampled row once a step). sink: device float[grid * 512], each
 * thread's sum of what it read (so the reads are used). layout 0: consecutive
 * lanes read consecutive 16-byte chunks of one row's piece (one instruction
 * covers whole pieces of a few rows); layout 1: the register tile's own lanes
 * (one instruction reads 64 bytes of each of 16 rows; a row's piece takes
 * several instructions; one row group, slices of at most 80 floats, eta <=
 * 1024, else RSK_ERR_UNSUPPORTED). An index outside [0, m) reads row 0.
 * Requires A float32, 16-byte aligned, n and ld multiples of 4, 1 <= eta <=
 * 4096, grid <= 1024 a multiple of row_groups.
 */
int32_t rsk_gather_rate_dense(const rsk_dense *A, const int32_t *index_stream, int32_t eta, int64_t K, int32_t grid,
                              int32_t row_groups, int32_t layout, float *sink, void *stream);

/* Version of this ABI (RSK_ABI_VERSION). */
int32_t rsk_abi_version(void);

/* Human-readable name of a status code (static string). */
const char *rsk_status_string(int32_t status);

/*
 * ||a_i||^2 of every row (the normalisation matrix D of Definition 1, squared).
 * rownorm2: device, m entries of A's dtype. Accumulates in double.
 */
int32_t rsk_rownorm2_dense(const rsk_dense *A, void *rownorm2, void *stream);
int32_t rsk_rownorm2_csr(const rsk_csr *A, void *rownorm2, void *stream);

/* Workspace bytes needed by the matching solve for this matrix and these parameters. */
int32_t rsk_workspace_size_dense(const rsk_dense *A, const rsk_params *p, size_t *bytes);
int32_t rsk_workspace_size_csr(const rsk_csr *A, const rsk_params *p, size_t *bytes);

/*
 * K steps of RSKA on a dense system (eq. (rska), Algorithm 1), in one
 * persistent launch.
 *   b       device, m entries.
 *   x_star  device, n entries, in/out: x*_K on return (read as x*_0 when warm_start = 1).
 *   x       device, n entries, out: S_lambda(x*_K).
 * Resuming: a call with warm_start = 1, the x_star of a previous call and
 * stream_offset advanced by K*eta continues that run exactly.
 * Kernels (p->kernel): 1 = general (float32 and float64, any alignment);
 * 2 = float32 register tile (n and ld multiples of 4, A 16-byte aligned,
 * eta <= 1024, slices of at most 80 columns); 3 = the register tile over two
 * row groups: each workgroup reads half of a step's rows over a slice twice
 * as wide (at most 160 columns), and the two workgroups of a slice add their
 * parts of the x* update in a third exchange (same requirements as 2, an
 * even number of workgroups); 4 = one workgroup of 256 threads with the
 * step in registers and no exchange between workgroups (float32 and float64,
 * any alignment; n <= 2048 and eta <= 32 / ceil-to-power-of-two(n / 256),
 * p->grid 0 or 1), the next step's rows loaded during the step: for small
 * systems, whose steps are bound by latency. 0 = the library's choice: for
 * float64 steps of at most 64 KB that kernel 4 takes, 4; for float32, 3 for
 * 88 <= eta <= 800 unless kernel 2's whole next-step tile fits its LDS
 * prefetch (one row pass of at most 9 float4 slots a thread), else 2, where
 * the register tile applies; else 1. The
 * kernels sum in different orders (results agree to rounding); each gives
 * bitwise reproducible x* and x (y_out: see rsk_params; kernel 4 applies y in
 * a fixed order as well).
 * A kernel that does not apply to the shape returns RSK_ERR_UNSUPPORTED.
 */
int32_t rsk_avg_solve_dense(const rsk_dense *A, const void *b, const rsk_params *p, void *x_star, void *x,
                            void *workspace, size_t ws_bytes, void *stream);

/*
 * rsk_avg_solve_dense for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same plan, kernels and results as rsk_avg_solve_dense, with
 * the cross-workgroup exchange words in a static device array of the library
 * (RSK_NOALLOC_SCRATCH_BYTES, 8 MiB, one copy per GPU, held until the process
 * ends) instead of a caller workspace. The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine); its scratch is cleared
 * by a fill kernel on `stream` before the solve. Arguments, device status and
 * errors as rsk_avg_solve_dense; a plan whose exchange needs more than the
 * static array (rsk_workspace_size_dense > RSK_NOALLOC_SCRATCH_BYTES) returns
 * RSK_ERR_WORKSPACE and queues nothing. Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (concurrent streams or host
 * threads) race and give undefined results; calls ordered on one stream are
 * safe. The address of the array is looked up on the first call on each device
 * (hipGetSymbolAddress, with that device current).
 */
#define RSK_NOALLOC_SCRATCH_BYTES (8u << 20)
int32_t rsk_avg_solve_dense_noalloc(const rsk_dense *A, const void *b, const rsk_params *p, void *x_star, void *x,
                                    void *stream);

/*
 * The launch rsk_avg_solve_dense would make for A and p, without making it
 * (nothing is queued; A->val is only inspected for its alignment). out:
 * host int32[9] = { kernel (1 general, 2 register tile, 3 register tile over
 * two row groups), workgroups G, threads per workgroup, row passes and float4
 * chunks per lane of the register tile (0 for the general kernel), row groups,
 * exchange hops per step (1 or 2), elements per vector load, row tile of the
 * general kernel (0 rows read from HBM twice a step, 1 one LDS tile, 2 two LDS
 * tiles with the next step's rows loaded during the step; 0 for the register
 * tile) }. Returns what rsk_avg_solve_dense would return for an unsupported
 * shape or bad argument.
 */
int32_t rsk_plan_dense(const rsk_dense *A, const rsk_params *p, int32_t *out);

/*
 * The same iteration with A in CSR form (eq. (rska) with sparse rows).
 * A sparse step moves a few hundred KB and is bound by latency. p->kernel
 * selects the kernel: 1 = one persistent workgroup (no cross-CU exchange),
 * 2 = the multi-workgroup kernel (one lane per nonzero, p->grid workgroups or
 * eta/8 up to the CU count, three grid barriers per step), 0 = 2 when
 * eta >= 4, else 1. Columns hit by several sampled rows of a step are summed
 * in int64 fixed point with a per-step power-of-two quantum (2^-41 of the
 * step's largest contribution), so x* and x are bitwise reproducible for a
 * given kernel (y_out: see rsk_params). eta <= 4096.
 * Workspace: n + 1 int64 accumulators, with y_out m int32 row counters (and
 * for the grid kernel eta coefficients), plus the grid kernel's barrier and
 * monitor words (rsk_workspace_size_csr, which depends on whether y_out is
 * set), zeroed by the call.
 * A column index outside [0, n) in a sampled row is RSK_ERR_INDEX_RANGE.
 */
int32_t rsk_avg_solve_csr(const rsk_csr *A, const void *b, const rsk_params *p, void *x_star, void *x,
                          void *workspace, size_t ws_bytes, void *stream);

/*
 * Many independent dense systems of uneven shape in one launch (eq. (rska)
 * per system, each with its own stream, eta, alpha, lambda, monitor, early
 * stop and status). System s runs on G_s workgroups, chosen so that each
 * holds about wg_bytes of the step's rows (at most 256); they split its
 * columns and exchange partial dots through the system's own workspace
 * region, exactly as rsk_avg_solve_dense does for one system. Persistent
 * workgroups take (system, rank) tickets in the order `order`. Two launches
 * exist: the general kernel (any dtype and alignment; 256-thread
 * workgroups, two a CU, the step's rows in LDS) and the float32 register
 * tile (512-thread workgroups, one a CU, the step's rows in VGPRs, column
 * slices of at most 160 floats, eta <= 512, every system's A 16-byte aligned
 * with ld % 4 == 0; a last float4 of a row that reaches past n reads the
 * row padding, which is masked to zero).
 *   nsys       number of systems (0 returns RSK_OK at once).
 *   dtype      RSK_F32 or RSK_F64, the dtype of every system.
 *   items      host array of nsys descriptors, checked before any launch
 *              (RSK_ERR_INVALID_ARG / RSK_ERR_UNSUPPORTED for the first bad one);
 *              it is not read after the call returns.
 *   items_dev  device copy of the same nsys descriptors; must stay valid until
 *              the stream has run the solve.
 *   order      device int32[nsys], a permutation of 0..nsys-1 (nullable: identity).
 *              Largest work first balances the CUs best. A repeated entry makes
 *              two groups write the same x (undefined result).
 *   wg_bytes   target row bytes per workgroup per step (0: the tuned class of
 *              the system's step bytes, else 56 KiB for the general kernel and
 *              256 KiB for the register tile). Must be the value given to
 *              rsk_workspace_size_batched.
 *   kernel     0: the register tile if every system takes it, else the general
 *              kernel; 1: general kernel; 2: register tile (RSK_ERR_UNSUPPORTED
 *              if a system does not fit it). Must be the value given to
 *              rsk_workspace_size_batched.
 * Per-system status_dev[0] is reset by the call; it ends 0 or an RSK_ERR_*
 * code, status_dev[1] the steps completed. The kernels plan from the device
 * copy: a device descriptor that is invalid or needs more LDS than the host
 * plan gives its system RSK_ERR_INVALID_ARG (the system is skipped); if the
 * device plans need more exchange words than the workspace holds, no system
 * runs and all report RSK_ERR_WORKSPACE.
 * Workspace: rsk_workspace_size_batched (plans, ticket counter and one
 * exchange region per system), zeroed by the call.
 */
int32_t rsk_workspace_size_batched(int32_t nsys, int32_t dtype, const rsk_batch_item *items, int64_t wg_bytes,
                                   int32_t kernel, size_t *bytes);
int32_t rsk_avg_solve_batched(int32_t nsys, int32_t dtype, const rsk_batch_item *items,
                              const rsk_batch_item *items_dev, const int32_t *order, int64_t wg_bytes,
                              int32_t kernel, void *workspace, size_t ws_bytes, void *stream);
/*
 * The launch rsk_avg_solve_batched would make (nothing is queued, no device
 * memory is touched): *kernel_out = 1 (general) or 2 (register tile), and
 * groups_out[i] = G_i, the workgroups of system i (host array of nsys).
 */
int32_t rsk_plan_batched(int32_t nsys, int32_t dtype, const rsk_batch_item *items, int64_t wg_bytes,
                         int32_t kernel, int32_t *kernel_out, int32_t *groups_out);

/*
 * Many right-hand sides sharing A and the index stream (float32 only), on the
 * matrix cores. Column r of X is the single-RHS iteration for b = B[:, r].
 * A step is the sketch-and-project form of the update (eq. (rska1), start of
 * Sec. 4) written as two GEMMs on the sampled rows A_tau:
 *     R = A_tau X - B_tau,  C = (alpha_k/eta) D_tau^-2 R,  X* -= A_tau^T C,  X = S_lambda(X*).
 *   B       device, m x R row-major.
 *   X_star  device, n x R row-major, in/out (read when warm_start = 1).
 *   X       device, n x R row-major, out.
 * Requires R % 4 == 0, n % 4 == 0, ld % 4 == 0, eta <= 4096, A 16-byte aligned; the
 * monitor and y_out are not supported here (RSK_ERR_UNSUPPORTED).
 * p->kernel: 1 = the step kernels (four launches per step, 64 x 64 product
 * tiles), 2 = one persistent cooperative launch for all K steps (the same
 * products and sums as the step kernels, tiles passed between workgroups
 * through device-coherent stores and per-tile counters), 3 = the step kernels
 * with wide product tiles (128 x 128 for A_tau X, 128 x 64 for the fused update
 * and whenever R <= 64; 512-thread workgroups; eta padded to a multiple of 128),
 * 0 = a tuned choice (rsk_tune_*), else 3 when R > 64 and eta >= 128, else 1.
 * Kernels 1 and 3 compute the same iteration with differently blocked sums
 * (equal to rounding).
 * Device faults and status_dev follow the single-RHS conventions (with kernel
 * 2, X* and X are unspecified after a fault).
 */
int32_t rsk_workspace_size_multirhs(const rsk_dense *A, int32_t R, const rsk_params *p, size_t *bytes);
int32_t rsk_avg_solve_multirhs(const rsk_dense *A, const void *B, int32_t R, const rsk_params *p, void *X_star,
                               void *X, void *workspace, size_t ws_bytes, void *stream);

/*
 * The split of rsk_avg_solve_multirhs's two products for A, R and p, without
 * running it. out: host int32[5] = { S: splits of the n columns in A_tau X
 * (fixed-order sum of S partials), columns per split, S2: splits of a step's
 * rows in A_tau^T C (1: one workgroup per output tile over all rows), eta
 * rounded up to a multiple of the tile edge (64, or 128 for kernel 3), the
 * kernel (1 step kernels, 2 one persistent launch, 3 wide-tile step kernels) }.
 */
int32_t rsk_plan_multirhs(const rsk_dense *A, int32_t R, const rsk_params *p, int32_t *out);

/*
 * rsk_avg_solve_multirhs that also writes the x* checkpoints the adjoint
 * recomputes from: before every step k with k % ckpt_every == 0, X* (n x R)
 * is copied to ckpt[k / ckpt_every]. ckpt: device, ceil(K / ckpt_every) x n x R
 * float32, caller-owned. Same workspace as rsk_avg_solve_multirhs.
 */
int32_t rsk_avg_solve_multirhs_ckpt(const rsk_dense *A, const void *B, int32_t R, const rsk_params *p,
                                    int32_t ckpt_every, void *X_star, void *X, void *ckpt, void *workspace,
                                    size_t ws_bytes, void *stream);

/*
 * Reverse mode of K unrolled multi-RHS RSKA steps (eq. (rska) with per-step
 * relaxation alpha_k, the iteration of Algorithm 1 differentiated step by
 * step). Given Xbar_K = dL/dx_K (n x R) for any loss L of x_K = S_lambda(x*_K),
 * computes
 *   Bbar       dL/dB (m x R, float32, overwritten),
 *   lambda_bar dL/dlambda (device double[1]),
 *   alpha_bar  dL/dalpha_k (device float32[K]),
 * with the subgradient of S_lambda taken as 1[|x*| > lambda] (0 at the kink).
 * The forward must have been run by rsk_avg_solve_multirhs_ckpt with the same
 * A, B, R, p and ckpt_every; X_star_K is its x*_K. Each segment of ckpt_every
 * steps is recomputed from its checkpoint (bitwise the forward's iterates),
 * then walked backwards: two float32 MFMA GEMMs per reverse step. Sums over
 * workgroups and repeated rows use fixed orders: results are reproducible.
 * p->alpha_k is required when K > 0; eta <= 4096; float32, R and n multiples of 4.
 * Workspace: rsk_workspace_size_adjoint.
 */
int32_t rsk_workspace_size_adjoint(const rsk_dense *A, int32_t R, const rsk_params *p, int32_t ckpt_every,
                                   size_t *bytes);
int32_t rsk_avg_adjoint(const rsk_dense *A, const void *B, int32_t R, const rsk_params *p, int32_t ckpt_every,
                        const void *ckpt, const void *X_star_K, const void *Xbar_K, void *Bbar, double *lambda_bar,
                        void *alpha_bar, void *workspace, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RSK_H */
