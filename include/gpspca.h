/*
 * gpspca.h -- C ABI of the MI355X (gfx950) implementation of the generalized
 * power method for sparse PCA (GP-SPCA).
 *
 * The method (paper, Section 2 and Table 1): for a data matrix A in R^{p x n}
 * (p samples in rows, n variables in columns a_i), find X on the unit sphere
 * (m = 1) or on the Stiefel manifold {X in R^{p x m} : X^T X = I_m} (block
 * forms, 1 <= m <= p) that maximizes one of the four reformulated objectives
 * of Table 1:
 *   SL1  F(x) = sum_i [ |a_i^T x| - gamma ]_+^2
 *   SL0  F(x) = sum_i [ (a_i^T x)^2 - gamma ]_+
 *   BL1  F(X) = sum_j sum_i [ mu_j |a_i^T x_j| - gamma ]_+^2
 *   BL0  F(X) = sum_j sum_i [ (mu_j a_i^T x_j)^2 - gamma ]_+
 * with t_+ = max(0, t).  Each iteration ("pass") computes the correlations
 * y_ij = a_i^T x_j, thresholds them (soft for l1: s = sign(y)[mu|y| - gamma]_+,
 * hard for l0: s = mu y where (mu y)^2 > gamma, else 0), forms the ascent
 * direction G = A S N (N = Diag(mu)), and retracts: x = g / ||g|| (m = 1) or
 * X = polar factor of G (block).  The sparse loadings of the original form
 * (Table 1, left column) are Z = S with unit-norm columns.
 *
 * Conventions shared by every entry point:
 *  - Device pointers are HIP device memory owned by the caller; host pointers
 *    are ordinary host memory.  The library keeps no pointer after a call
 *    returns.
 *  - Matrices are column-major.  A is p x n with leading dimension lda >= p.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is stream-ordered; calls that return host results synchronize the
 *    stream before returning.
 *  - gamma is absolute and the same for every component; mu (block forms
 *    only, host, m entries, NULL = all ones) must be positive and finite.
 *  - The return value is a status: 0 OK, > 0 outputs valid but flagged,
 *    < 0 error (outputs unspecified).  No exception or abort crosses the ABI.
 *    gpspca_last_error() gives a message for the calling thread.
 *  - Arguments are validated on the host before any HIP call.
 *  - The solve path never allocates device memory: all scratch lives in a
 *    caller-provided workspace of gpspca_workspace_bytes() bytes.
 */
#ifndef GPSPCA_H
#define GPSPCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Formulations (Table 1). */
#define GPSPCA_SL1 0
#define GPSPCA_SL0 1
#define GPSPCA_BL1 2
#define GPSPCA_BL0 3
/* Block L1 read from its original form (Table 1, left column): for fixed X the
 * maximum over unit-norm z_j of mu_j x_j^T A z_j - gamma ||z_j||_1 is ||s_j||,
 * so F(X) = sum_j ||s_j|| = sum_j sqrt(sum_i [mu_j |a_i^T x_j| - gamma]_+^2) and
 * the ascent direction is column j of A S N divided by ||s_j||.  The pass is
 * BL1's; the objective and the retraction X = polar(A S N Diag(1/||s_j||))
 * differ for m > 1 (for m = 1 the iterates are SL1's and F is the square root
 * of SL1's).  Accepted by gpspca_workspace_bytes and gpspca_solve only. */
#define GPSPCA_BL1X 4

/* Storage types of A.  The paper stores A in full precision; 16- and 8-bit
 * storage is an extension that moves 2 or 1 bytes per element per pass while
 * the arithmetic stays FP32 (see gpspca_quantize for the rounding). */
#define GPSPCA_F32 0
#define GPSPCA_BF16 1     /* bfloat16 codes; value = bf16 * col_scale[i] (scale optional);
                             lda a multiple of 8, data 16-byte aligned */
#define GPSPCA_F8E4M3 2   /* OCP float8 e4m3fn codes; value = e4m3 * col_scale[i] (scale
                             required); lda a multiple of 16, data 16-byte aligned */

/* Status codes. */
#define GPSPCA_OK 0
#define GPSPCA_MAXITER 1      /* stopped at max_iter before the tolerance test held */
#define GPSPCA_DEGENERATE 2   /* some component had an empty support (completed), or F = 0 */
#define GPSPCA_EINVAL (-1)    /* invalid argument, or a rank-deficient starting point */
#define GPSPCA_EDTYPE (-2)    /* unsupported storage type for this call */
#define GPSPCA_ENOMEM (-3)    /* workspace (or server arena) too small */
#define GPSPCA_EDEVICE (-4)   /* a HIP runtime error */
#define GPSPCA_ENONFINITE (-5)/* the objective or the ascent direction became non-finite */

/* Largest number of components handled by the block kernels. */
#define GPSPCA_MAX_M 64

/* A data matrix (Section 2: p samples x n variables). */
typedef struct gpspca_matrix {
    const void* data;        /* device, column-major p x n */
    int64_t p;               /* rows (samples), >= 1 */
    int64_t n;               /* columns (variables), 1 <= n < 2^31 */
    int64_t lda;             /* leading dimension in elements, >= p */
    int32_t dtype;           /* GPSPCA_F32 | GPSPCA_BF16 | GPSPCA_F8E4M3 */
    int32_t reserved;
    const float* col_scale;  /* device, n FP32 per-column scales (BF16: optional, F8E4M3:
                                required, F32: must be NULL) */
} gpspca_matrix;

/* Bytes of device workspace that gpspca_solve needs for this problem.
 * Returns 0 if the arguments are invalid (see gpspca_last_error()). */
size_t gpspca_workspace_bytes(const gpspca_matrix* A, int form, int m, int max_iter);

/*
 * Solve one GP-SPCA problem by the power iteration (Section 2, Table 1).
 *
 *  A          data matrix (F32, BF16 or F8E4M3 storage; FP32 arithmetic).
 *  form       GPSPCA_SL1 | SL0 (then m must be 1) | BL1 | BL0 | BL1X
 *             (1 <= m <= min(p, 64)).
 *  gamma      absolute sparsity weight >= 0.
 *  mu         host, m weights > 0 for block forms; NULL = all ones; ignored for SL*.
 *  X0         device p x m starting point (leading dim p), or NULL for the default
 *             start: the m columns of A with the largest norms (ties to the lower
 *             index).  The start is projected onto the feasible set (normalized or
 *             polar factor); a rank-deficient start returns GPSPCA_EINVAL.
 *  tol        stop when |F_k - F_{k-1}| < tol * |F_{k-1}| (k >= 1); 0 = never.
 *  max_iter   maximum number of passes (>= 1).
 *  workspace  device, ws_bytes >= gpspca_workspace_bytes(A, form, m, max_iter),
 *             256-byte aligned.
 * Outputs (device unless noted; any except X may be NULL):
 *  X          p x m (leading dim p): X_k, the iterate of the last pass.
 *  Z          n x m (leading dim n): thresholded correlations of the last pass with
 *             unit-norm columns (a column with empty support is all zeros).
 *  support    ceil(n/32) x m uint32 words: bit (i % 32) of word (j * ceil(n/32) + i/32)
 *             is set iff Z[i, j] != 0.
 *  obj_trace  host, max_iter doubles: F_0 .. F_{n_iter-1}.
 *  n_iter     host: number of passes made.
 * The iteration stops at pass k when F_k = 0, when the tolerance test holds, or
 * when k + 1 = max_iter.  After an error status (< 0) the device outputs hold
 * unspecified values.  Synchronizes `stream` before returning.
 */
int gpspca_solve(const gpspca_matrix* A, int form, int m, double gamma, const double* mu,
                 const float* X0, double tol, int max_iter,
                 void* workspace, size_t ws_bytes, void* stream,
                 float* X, float* Z, uint32_t* support, double* obj_trace, int* n_iter);

/* Size of the library's own device scratch for gpspca_solve_noalloc (bytes). */
#define GPSPCA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * gpspca_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, and harnesses that forbid hipMalloc.  The
 * iteration, arguments, outputs and statuses are gpspca_solve's; in place of a
 * caller workspace the call uses a scratch array that the library holds in
 * device memory, GPSPCA_NOALLOC_SCRATCH_BYTES per GPU (each GPU the library
 * runs on keeps its own copy until the process ends).  The call allocates
 * nothing: no hipMalloc, hipFree, pinned host memory, events or graphs (its
 * passes are enqueued one by one).
 *  - A problem whose scratch (its gpspca_workspace_bytes for the default
 *    kernel configuration) exceeds GPSPCA_NOALLOC_SCRATCH_BYTES is rejected with
 *    GPSPCA_ENOMEM before any device work.
 *  - Every call on one GPU uses that GPU's one scratch array, and each call
 *    initializes what it reads: calls that overlap on one GPU (other host
 *    threads, or other streams of this call's device) race and must be
 *    serialized by the caller.
 * Synchronizes `stream` before returning.
 */
int gpspca_solve_noalloc(const gpspca_matrix* A, int form, int m, double gamma,
                         const double* mu, const float* X0, double tol, int max_iter,
                         void* stream, float* X, float* Z, uint32_t* support,
                         double* obj_trace, int* n_iter);

/*
 * One pass of the iteration at a given feasible point X (device p x m, leading
 * dim p, used as given: it is not re-projected).  For step-level checks.
 * Outputs: S (device n x m, leading dim n): thresholded correlations;
 * G (device p x m doubles, leading dim p): G = A S Diag(mu);
 * f (host, m doubles): per-component objective terms (F = sum_j f_j);
 * nnz (host, m int64): per-component support sizes.
 * Uses the same workspace as gpspca_solve (max_iter = 1).  Synchronizes.
 */
int gpspca_step(const gpspca_matrix* A, int form, int m, double gamma, const double* mu,
                const float* X, void* workspace, size_t ws_bytes, void* stream,
                float* S, double* G, double* f, int64_t* nnz);

/*
 * Gamma path: K independent single-unit problems on the same A (Table 1, SL1
 * or SL0), problem k with its own sparsity weight gammas[k].  Every pass over A
 * serves all K problems (the correlations of the K columns of X come from one
 * read of A); each column is retracted on its own sphere (x_k = g_k/||g_k||) and
 * has its own stopping rule, after which it is frozen, so column k's result is
 * that of gpspca_solve(A, form, 1, gammas[k], ...) from the same start.
 *
 *  K          1 <= K <= GPSPCA_MAX_M problems.
 *  gammas     host, K absolute weights >= 0.
 *  X0         device p x K starts (leading dim p; each column is normalized), or
 *             NULL: every column starts at the normalized column of largest norm.
 *  workspace  >= gpspca_path_workspace_bytes(A, K, max_iter) bytes, 256-aligned.
 * Outputs: X (device p x K), Z (device n x K), support (device ceil(n/32) x K
 * words) as in gpspca_solve; obj_trace (host, K x max_iter doubles, problem k's
 * trace at obj_trace[k * max_iter ...]); n_iter and status (host, K ints).
 * Returns GPSPCA_OK when every problem converged, otherwise the largest
 * per-problem status (or a negative error).  Synchronizes `stream`.
 */
size_t gpspca_path_workspace_bytes(const gpspca_matrix* A, int K, int max_iter);
int gpspca_solve_path(const gpspca_matrix* A, int form, int K, const double* gammas,
                      const float* X0, double tol, int max_iter,
                      void* workspace, size_t ws_bytes, void* stream,
                      float* X, float* Z, uint32_t* support, double* obj_trace,
                      int* n_iter, int* status);

/*
 * Multi-start single-unit solves: m independent problems of one single-unit
 * formulation (form GPSPCA_SL1 or GPSPCA_SL0) with the same gamma, problem k
 * starting at the column of A with the k-th largest norm (ties to the lower
 * index), normalized.  They share every pass over A exactly as the problems of
 * gpspca_solve_path do (Section 2, Table 1, rows 1-2, run from m starts: the
 * reading of "m" for single-unit serving requests).  1 <= m <= min(n,
 * GPSPCA_MAX_M).  Workspace: gpspca_path_workspace_bytes(A, m, max_iter).
 * Outputs, return value and synchronization as in gpspca_solve_path with K = m.
 */
int gpspca_solve_multistart(const gpspca_matrix* A, int form, int m, double gamma, double tol,
                            int max_iter, void* workspace, size_t ws_bytes, void* stream,
                            float* X, float* Z, uint32_t* support, double* obj_trace,
                            int* n_iter, int* status);

/*
 * m sparse components of a single-unit formulation (form GPSPCA_SL1 or
 * GPSPCA_SL0, Section 2, Table 1, rows 1-2) by projection deflation: component
 * k is the single-unit solve on A_k = (I - Q Q^T) A, Q = [x_0 .. x_{k-1}] the
 * components already found, from the default start of A_k (its column of
 * largest norm, ties to the lower index, normalized).  The paper reports
 * single-unit timings for several components (Section 4.1) without fixing how
 * they are obtained; deflation of the data matrix is the reading taken here.
 * A_k is never formed: A_k^T x = A^T x for x in the range of I - Q Q^T, so each
 * pass runs on A and the new iterate is projected back, x <- P x / ||P x||, in
 * FP64 (P = I - Q Q^T).  FP32 storage only.
 *
 *  m          1 <= m <= min(p, n, GPSPCA_MAX_M) components.
 *  gamma      absolute weight >= 0, the same for every component.
 *  workspace  >= gpspca_deflated_workspace_bytes(A, m, max_iter) bytes,
 *             256-aligned (device; holds Q in FP64 besides one solve's memory).
 * Outputs: X (device p x m, leading dim p), Z (device n x m), support (device
 * ceil(n/32) x m words) as in gpspca_solve, component k in column k;
 * obj_trace (host, m x max_iter doubles, component k's trace at
 * obj_trace[k * max_iter ...], n_iter[k] entries valid); n_iter and status
 * (host, m ints).  Returns GPSPCA_OK when every component converged, the
 * largest per-component status otherwise, or a negative error (EDTYPE for
 * 16/8-bit storage; EINVAL when A_k is zero, i.e. the rank of A is below
 * k + 1: components 0 .. k-1 are then already written).  Synchronizes
 * `stream`.
 */
size_t gpspca_deflated_workspace_bytes(const gpspca_matrix* A, int m, int max_iter);
int gpspca_solve_deflated(const gpspca_matrix* A, int form, int m, double gamma, double tol,
                          int max_iter, void* workspace, size_t ws_bytes, void* stream,
                          float* X, float* Z, uint32_t* support, double* obj_trace,
                          int* n_iter, int* status);

/*
 * Refinement on a frozen support (for results of a reduced-precision solve).
 * Runs passes of the iteration of gpspca_solve on the FP32 matrix A in which
 * s_ij is forced to 0 wherever bit (i % 32) of word (j * ceil(n/32) + i/32) of
 * `support_in` (device, as written by gpspca_solve) is clear; only the
 * columns with a bit set are read.  X0 (device p x m, required) is the start,
 * typically the reduced-precision result; it is projected like gpspca_solve's
 * X0.  tol, max_iter, the workspace (gpspca_workspace_bytes of the same
 * problem) and the outputs are those of gpspca_solve.  A must be F32
 * (GPSPCA_EDTYPE otherwise).  Synchronizes `stream`.
 */
int gpspca_refine(const gpspca_matrix* A, int form, int m, double gamma, const double* mu,
                  const uint32_t* support_in, const float* X0, double tol, int max_iter,
                  void* workspace, size_t ws_bytes, void* stream,
                  float* X, float* Z, uint32_t* support, double* obj_trace, int* n_iter);

/* The same for a gamma path: K single-unit problems, problem k restricted to
 * its own support words (k * ceil(n/32) ...), started from column k of X0.
 * Workspace: gpspca_path_workspace_bytes(A, K, max_iter).  Outputs as in
 * gpspca_solve_path. */
int gpspca_refine_path(const gpspca_matrix* A, int form, int K, const double* gammas,
                       const uint32_t* support_in, const float* X0, double tol, int max_iter,
                       void* workspace, size_t ws_bytes, void* stream,
                       float* X, float* Z, uint32_t* support, double* obj_trace,
                       int* n_iter, int* status);

/*
 * Reduced-precision copy of an FP32 matrix A (device) into `out` (device,
 * column-major, leading dimension ldq >= p elements; ldq a multiple of 8 for
 * BF16 and of 16 for F8E4M3 if the result is to be solved on; rows p..ldq-1 are
 * left untouched).
 *  to = GPSPCA_BF16:    out = bfloat16(a_ri), rounded to nearest even; if
 *                       col_scale is not NULL it receives n ones.
 *  to = GPSPCA_F8E4M3:  col_scale[i] = max_r |a_ri| / 448 in FP32 (1 for a
 *                       zero column); out = e4m3fn(a_ri / col_scale[i]) rounded
 *                       to nearest even and saturated at +-448 (col_scale
 *                       required, device, n floats).
 * Stream-ordered; does not synchronize.
 */
int gpspca_quantize(const gpspca_matrix* A, int to, void* out, int64_t ldq, float* col_scale,
                    void* stream);

/*
 * Autotuner of the correlation kernel.  Times every candidate configuration
 * for this problem (kernel variant: LDS-staged or register-direct matrix-core
 * kernel, or X-in-registers VALU kernel; LDS stages; workgroups per CU) over
 * `passes` passes of the iteration from the feasible start X0 (device p x m,
 * leading dim p), and records the fastest in a process-wide table (thread-safe)
 * that every later plan with the same storage type, m, p, n, alignment and kind
 * (single problem, or a gamma path when form is SL1/SL0 and m > 1) uses.
 * Environment overrides (GPSPCA_CORR_KERNEL, GPSPCA_MFMA_STAGES,
 * GPSPCA_MFMA_WAVES_PER_CU) still take precedence.  Configurations whose
 * workspace exceeds ws_bytes are skipped; gpspca_workspace_bytes (or
 * gpspca_path_workspace_bytes) covers all of them.  A tuned configuration
 * changes results only within FP32 rounding (every configuration reduces in a
 * fixed order, so each is deterministic).  Outputs (host, may be NULL): the
 * number of configurations timed, the best time per pass (ms) and a short
 * description of the chosen configuration.  Synchronizes `stream`.
 */
int gpspca_autotune(const gpspca_matrix* A, int form, int m, double gamma, const float* X0,
                    int passes, void* workspace, size_t ws_bytes, void* stream,
                    int* n_timed, double* best_ms, char* best_desc, size_t desc_len);
/* Forget every tuned configuration (later plans use the defaults again). */
int gpspca_autotune_clear(void);

/*
 * Column norms ||a_i||_2 of A (FP64 accumulation) into device `norms` (n doubles).
 * Stream-ordered; does not synchronize.
 */
int gpspca_column_norms(const gpspca_matrix* A, double* norms, void* stream);

/* ------------------------------------------------------------------------
 * Solve server: continuous batching of independent solves on one GPU.
 *
 * The method solves one problem at a time; a service answers many, on many
 * matrices.  The server keeps `slots` solves in flight (one HIP stream and one
 * host worker thread each), admitting a waiting request as soon as a slot and
 * device memory are free, so requests that arrive while others run overlap on
 * the device.  All device memory comes from one caller-provided arena (device,
 * 256-byte aligned, owned by the caller until gpspca_server_destroy returns):
 * 64 MB of upload staging per slot, the rest shared by resident matrices and
 * per-request workspaces.  A matrix is uploaded (host to device) on the first
 * admitted request that needs it and stays resident, with its column norms, for
 * later requests; when memory is needed, resident matrices that no admitted
 * request uses are evicted, least recently used first.  Admission is in arrival
 * order, except that a request that does not fit yet may be passed by later
 * ones a bounded number of times.  Every result equals what gpspca_solve
 * returns for the same problem from the default start; a single-unit request
 * with m > 1 is m starts, as gpspca_solve_multistart.
 * ------------------------------------------------------------------------ */
typedef struct gpspca_server gpspca_server;

typedef struct gpspca_result {
    int status;               /* status of the solve (as gpspca_solve) */
    int n_iter;
    int m;
    int uploaded;             /* 1 if this request uploaded its matrix */
    int64_t p, n;
    const float* X;           /* host p x m (leading dim p), owned by the server */
    const float* Z;           /* host n x m */
    const uint32_t* support;  /* host ceil(n/32) x m words, as gpspca_solve */
    const double* obj_trace;  /* host n_iter entries (multi-start: m x n_iter, problem k's
                                 trace at obj_trace[k * n_iter], col_n_iter[k] entries) */
    double t_submit, t_admit, t_done;  /* seconds since the server was created */
    const int* col_n_iter;    /* multi-start: per-problem passes (n_iter is their max); else NULL */
    const int* col_status;    /* multi-start: per-problem status (status is the largest); else NULL */
} gpspca_result;

typedef struct gpspca_stats {
    int64_t waiting, running, completed, uploads, evictions;
    size_t resident_bytes, free_bytes, arena_bytes;
} gpspca_stats;

/* slots: 1..16 concurrent solves.  arena_bytes >= slots * 64 MB + 64 MB. */
int gpspca_server_create(void* arena, size_t arena_bytes, int slots, gpspca_server** out);
/* Register a host FP32 matrix (p x n, column-major, leading dim ld >= p) that the
 * caller keeps unchanged until it is unregistered; store_dtype GPSPCA_F32 or
 * GPSPCA_BF16 (quantized on the device at upload, as gpspca_quantize). */
int gpspca_server_register(gpspca_server* s, const float* host, int64_t p, int64_t n, int64_t ld,
                           int store_dtype, uint64_t* matrix_id);
/* Fails while the matrix has pending requests. */
int gpspca_server_unregister(gpspca_server* s, uint64_t matrix_id);
/* Queue a solve (arguments as gpspca_solve, default start; a single-unit form
 * with m > 1 as gpspca_solve_multistart); returns at once.  GPSPCA_ENOMEM if
 * the request could not fit even in an empty arena. */
int gpspca_server_submit(gpspca_server* s, uint64_t matrix_id, int form, int m, double gamma,
                         const double* mu, double tol, int max_iter, uint64_t* request_id);
/* 0 and *out filled when the request is done, 1 while it is pending, < 0 on
 * error.  The result's arrays stay valid until gpspca_server_release. */
int gpspca_server_poll(gpspca_server* s, uint64_t request_id, gpspca_result* out);
/* Blocks until the request is done, then as gpspca_server_poll. */
int gpspca_server_wait(gpspca_server* s, uint64_t request_id, gpspca_result* out);
/* Frees a finished request's host results. */
int gpspca_server_release(gpspca_server* s, uint64_t request_id);
int gpspca_server_stats(gpspca_server* s, gpspca_stats* out);
/* Waits for every submitted request, stops the workers and frees the server
 * (the arena is the caller's again). */
int gpspca_server_destroy(gpspca_server* s);

/* Message describing the last non-OK status returned on the calling thread. */
const char* gpspca_last_error(void);

/* Library version string. */
const char* gpspca_version(void);

/*
 * Kernel timing for roofline reports.  While enabled (on >= 1), the solve path
 * times launches of its dominant (A-streaming) correlation kernel with a pair
 * of HIP events that the launch itself records at the kernel's start and end
 * (hipExtLaunchKernelGGL): the first launch of each solve and every on-th one
 * after it (on = 1: every launch).  on <= 0 disables timing.
 * gpspca_profile_read returns the summed duration (ms) of the timed launches,
 * their count, and the name of the kernel, then resets the counters.  Solves
 * whose correlation runs as several launches (the vector-ALU fallback for
 * unaligned A) report no timed launches.
 */
int gpspca_profile_enable(int on);
int gpspca_profile_read(double* total_ms, int64_t* launches, char* name, size_t name_len);

#ifdef __cplusplus
}
#endif
#endif /* GPSPCA_H */
