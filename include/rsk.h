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

#define RSK_ABI_VERSION 1

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
  void *y_out;                 /* nullable device array (m, dtype of A), in/out: y[tau_t] -= c_t, so x* = A^T y */
  int32_t *status_dev;         /* device int32[2]: [0] status (0 = ok), [1] steps completed. Required. */
  int32_t grid;                /* workgroups of the persistent kernel; 0 = chosen by the library */
  int32_t kernel;              /* dense kernel: 0 = chosen by the library, 1 = general, 2 = float32 register tile */
} rsk_params;

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
 */
int32_t rsk_avg_solve_dense(const rsk_dense *A, const void *b, const rsk_params *p, void *x_star, void *x,
                            void *workspace, size_t ws_bytes, void *stream);

/*
 * The same iteration with A in CSR form (eq. (rska) with sparse rows).
 * Runs as one persistent workgroup: a sparse step moves a few hundred KB
 * and is bound by latency, which a single CU minimises (no cross-CU exchange).
 * Columns hit by several sampled rows of a step are summed in int64 fixed
 * point with a per-step power-of-two quantum (2^-41 of the step's largest
 * contribution), so results are bitwise reproducible. eta <= 4096.
 * Workspace: n int64 accumulators (rsk_workspace_size_csr), zeroed by the call.
 * A column index outside [0, n) in a sampled row is RSK_ERR_INDEX_RANGE.
 */
int32_t rsk_avg_solve_csr(const rsk_csr *A, const void *b, const rsk_params *p, void *x_star, void *x,
                          void *workspace, size_t ws_bytes, void *stream);

/*
 * Many right-hand sides sharing A and the index stream (float32 only), on the
 * matrix cores. Column r of X is the single-RHS iteration for b = B[:, r].
 * A step is the sketch-and-project form of the update (eq. (rska1), start of
 * Sec. 4) written as two GEMMs on the sampled rows A_tau:
 *     R = A_tau X - B_tau,  C = (alpha_k/eta) D_tau^-2 R,  X* -= A_tau^T C,  X = S_lambda(X*).
 *   B       device, m x R row-major.
 *   X_star  device, n x R row-major, in/out (read when warm_start = 1).
 *   X       device, n x R row-major, out.
 * Requires R % 4 == 0, n % 4 == 0, ld % 4 == 0, A 16-byte aligned; the
 * monitor and y_out are not supported here (RSK_ERR_UNSUPPORTED).
 * Device faults and status_dev follow the single-RHS conventions; steps are
 * queued as kernels on `stream` (four per step).
 */
int32_t rsk_workspace_size_multirhs(const rsk_dense *A, int32_t R, const rsk_params *p, size_t *bytes);
int32_t rsk_avg_solve_multirhs(const rsk_dense *A, const void *B, int32_t R, const rsk_params *p, void *X_star,
                               void *X, void *workspace, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RSK_H */
