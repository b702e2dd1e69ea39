/*
 * gap.h -- C ABI of the MI355X (gfx950) sparse-GP (GAP) fit library.
 *
 * The library fits the weights c of a sparse Gaussian-process model of total
 * energies (Sec. Theory of "Massively Parallel Fitting of Gaussian
 * Approximation Potentials"):
 *
 *   E_A = sum_{i in A} eps(x_i),  eps(x) = sum_j c_j k(x, x_j)     (Eqs. 1-2)
 *   k(x, x') = sigma_w^2 (x . x')^zeta   (dot-product covariance, integer zeta)
 *   minimise L(c) = (y - K_NM c)^T Sigma^-1 (y - K_NM c) + c^T K_MM c  (Eq. loss)
 *
 * by the stable route of Sec. Theory: K_MM (+ jitter on its diagonal) =
 * L L^T, A = [Sigma^-1/2 K_NM ; L^T] ((N+M) x M), b = [Sigma^-1/2 y ; 0],
 * A = QR by Householder reflections, c = R^-1 Q^T b.
 *
 * Conventions for every entry point:
 *  - Pointers named x_*, config_offsets, sigma, y, c, c_out, y_out and the
 *    workspace are DEVICE pointers (HBM of the GPU current when the handle was
 *    created), owned by the caller; the library never allocates device memory
 *    and never frees what it is given.  gap_params, gap_solve_info and
 *    gap_layout_info are host structs.
 *  - Work is enqueued asynchronously on the handle's HIP stream (a hipStream_t
 *    passed as void*; NULL = the default stream).  Inputs must stay valid and
 *    unmodified until that work completes; sigma given to gap_build_knm is
 *    read again by gap_solve (b assembly) and must stay valid until gap_solve's
 *    work completes; the sparse set given to gap_build_knm must stay valid for
 *    later gap_predict calls.
 *  - Argument errors are detected synchronously, before anything is enqueued,
 *    and returned as GAP_EINVAL / GAP_ENOMEM / GAP_ESTATE.  Failures found on
 *    the device (Cholesky pivot not positive, non-finite values) are reported
 *    through gap_solve_info.device_status and the status returned by
 *    gap_solve (when it is given an info struct) or gap_sync.
 *  - A handle is used from one host thread at a time; independent handles
 *    may run concurrently on different streams.
 *  - Call order: gap_create -> gap_bind_workspace -> gap_build_knm ->
 *    gap_solve -> gap_predict*; gap_build_knm may be called again to start a
 *    new fit in the same handle.  Batched: gap_build_knm_batch over several
 *    handles, then gap_build_kmm on each, then gap_solve.  A predict-only
 *    handle: gap_create -> gap_set_model -> gap_predict*.
 *  - Descriptors are used as given: the covariance assumes unit-L2 rows but
 *    does not renormalise them.
 */
#ifndef GAP_H
#define GAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gap_status {
    GAP_OK = 0,
    GAP_EINVAL = 1,      /* bad argument: shape, pointer, zeta outside 1..8, sigma_w <= 0 */
    GAP_ENOMEM = 2,      /* the bound workspace is smaller than gap_workspace_bytes() */
    GAP_ENOTPD = 3,      /* K_MM + jitter is not positive definite (Cholesky pivot <= 0) */
    GAP_ENONFINITE = 4,  /* a NaN or Inf reached the weights */
    GAP_ENOCONV = 5,     /* mixed precision: refinement did not converge within max_refine_iters */
    GAP_EDEVICE = 6,     /* a HIP runtime call failed, or a device-side wait was abandoned */
    GAP_ESTATE = 7,      /* entry points called out of order */
    GAP_ERANK = 8        /* the stacked matrix is numerically rank deficient (a QR panel's
                            Gram matrix lost positive definiteness even with the shift) */
} gap_status;

typedef enum gap_precision {
    GAP_FP64 = 0,        /* every stage in FP64 */
    GAP_MIXED_FP32 = 1,  /* FP64 K_NM/Cholesky; FP32 Householder QR with FP64 reflector norms;
                            FP64 iterative refinement of c against the FP64 A: corrected
                            semi-normal equations preconditioned by the FP32 R, moving to
                            R-preconditioned CGLS when a correction fails to halve (A too
                            ill-conditioned for FP32, kappa(A) near 1/u_32 or above).
                            The factored FP32 matrix is the FP64 A rounded to FP32. */
    GAP_MIXED_BF16 = 2,  /* as GAP_MIXED_FP32, but the factored matrix's K_NM block comes from
                            descriptor dot products on BF16 MFMA (descriptors rounded to BF16,
                            FP32 accumulation), with the power, the per-configuration sums and
                            the row scale in FP32.  The FP64 K_NM is built as well: the
                            refinement's residuals use the FP64 A, so c converges to the FP64
                            problem's solution (or the status is GAP_ENOCONV). */
    GAP_MIXED_FP16 = 3   /* as GAP_MIXED_BF16 with FP16 descriptors and FP16 MFMA */
} gap_precision;

/* Fit parameters (host struct). */
typedef struct gap_params {
    int32_t d;                /* descriptor length, >= 1 */
    int32_t zeta;             /* kernel exponent, 1..8 */
    double sigma_w;           /* kernel prefactor sigma_w (> 0); k carries sigma_w^2 */
    double jitter;            /* added to K_MM's diagonal before the Cholesky (>= 0) */
    int32_t precision;        /* gap_precision */
    int32_t max_refine_iters; /* mixed precision only: refinement iteration cap (both stages) */
    double refine_tol;        /* mixed precision only: stop when a step's ||dc||/||c|| <= refine_tol,
                                 or when ||dc|| stops halving at a level <= 1e-9 ||c|| (FP64
                                 rounding floor) */
    uint32_t flags;           /* GAP_FLAG_* */
} gap_params;

/* Record per-stage durations with HIP events (read back by gap_stage_times). */
#define GAP_FLAG_TIMING 1u
/* Estimate the relative error of c (gap_solve_info.est_err): 16 steps each of
 * power and inverse iteration on R for kappa_2(A), about 32 triangular solves. */
#define GAP_FLAG_ERROR_ESTIMATE 2u
/* Build the FP64 K_NM from descriptor dot products emulated on INT8 MFMA
 * (Ozaki scheme; the K_MN definition of Sec. Theory): every descriptor and
 * sparse row is scaled by a power of two and rounded to a 54-bit integer, split
 * into 7 signed 8-bit slices, and the 28 leading slice products are summed
 * exactly in INT32 and combined in FP64 (the power, segment sums and row scale
 * in FP64 as in the FP64 build).  The dot products carry about FP64's rounding
 * error.  Applies to every precision (the FP64 A of the mixed forms included);
 * K_MM keeps the FP64 build.  The workspace grows by 7 bytes per descriptor
 * entry (rows padded to a multiple of 32) plus 4 bytes per row.  Parameters
 * with this flag and d > 4096 are rejected (GAP_EINVAL, or 0 workspace bytes):
 * beyond that the INT32 sums could overflow. */
#define GAP_FLAG_KNM_INT8 4u
/* Checking aid (not for production runs): at the start of every build, fill
 * every floating-point and descriptor-slice array of the workspace with
 * all-ones bytes (a NaN in FP64, FP32, BF16 and FP16; -1 in the INT8 slices
 * and INT32 exponents) before the build writes it.  A read of workspace memory
 * that the build or the solve did not write first then turns into a
 * non-finite or wrong result that the parity tests see.  The tile plans,
 * counters, status words and flags are not filled: the build clears or writes
 * them itself, and they hold indices and loop bounds.  Costs one pass over
 * those arrays per build. */
#define GAP_FLAG_POISON_WORKSPACE 8u

typedef struct gap_handle_s *gap_handle;

typedef struct gap_solve_info {
    int32_t device_status;   /* gap_status found on the device (GAP_OK when none) */
    int32_t refine_iters;    /* mixed precision: refinement iterations done (0 in FP64) */
    double residual_norm2;   /* min of the loss at the returned c: ||(Q^T b)[M:]||^2 in FP64,
                                ||b - A c||^2 against the FP64 A in mixed precision */
    double grad_rel;         /* normal-equation residual (zero gradient of Eq. loss, Eq. GP_sparse)
                                of the returned c: ||A^T (b - A c)|| / (||A||_F (||A||_F ||c|| + ||b||)).
                                Mixed precision: against the FP64 A.  FP64: in the factored basis,
                                A^T r = R^T ((Q^T b)[0:M] - R c), which checks the back-substitution
                                (the QR's own backward error, about u, is not included) */
    int32_t cgls_iters;      /* mixed precision: how many of refine_iters were preconditioned
                                CGLS steps (0 when the corrected semi-normal equations converged) */
    int32_t reserved;        /* 0 */
    double step_rel;         /* mixed precision: the last refinement step's ||dc|| / ||c||; 0 in FP64 */
    double est_err;          /* with GAP_FLAG_ERROR_ESTIMATE: estimated relative error of c,
                                u (kappa + kappa^2 ||r|| / (||A||_2 ||c||)), u = 2^-53, kappa =
                                kappa_2(A) from power / inverse iteration on R (the FP32 R in mixed
                                precision); -1 when not requested */
    double kappa_est;        /* the kappa_2(A) estimate behind est_err (0 when not requested) */
} gap_solve_info;

/* Where the library keeps its stage outputs inside the bound workspace (host struct).
 * A_aug is column-major with leading dimension lda (in elements):
 *   rows 0..N-1, cols 0..M-1      Sigma^-1/2 K_NM after gap_build_knm; R and reflectors after gap_solve
 *   rows N..N+M-1, cols 0..M-1    L^T (upper triangular) after gap_build_knm
 *   col M                          b = [Sigma^-1/2 y ; 0] during gap_solve, Q^T b after it
 *   rows N+M..lda-1 are unused padding (never read). */
typedef struct gap_layout_info {
    double *A_aug;
    int64_t lda;          /* rows of A_aug in memory (>= N + M) */
    int64_t ncols;        /* columns of A_aug in memory (>= M + 1) */
    int64_t N, M, n_atoms;
    double *tau;          /* [M] Householder weights after gap_solve */
    int32_t *device_status;
    float *A32;           /* mixed precision: FP32 copy of [A | b] (same lda), holding R,
                             reflectors and Q^T b after gap_solve; NULL in FP64 */
} gap_layout_info;

/* Create a handle bound to the current HIP device and `stream` (hipStream_t or NULL).
 * Validates p (GAP_EINVAL).  Allocates only host memory and HIP events.  The
 * first gap_build_knm of a fit that uses the QR look-ahead (gap_tuning) also
 * creates one internal HIP stream (default priority) and its events; make that
 * first call outside graph capture.  Inside gap_build_knm / gap_build_knm_obs
 * (K_MM and its Cholesky, beside the K_NM) and gap_solve (the QR's trailing
 * updates) that stream forks from and joins `stream`, so a graph captured on
 * `stream` contains it and the calls' work is complete when `stream`'s is. */
gap_status gap_create(const gap_params *p, void *stream, gap_handle *out);

/* Bytes of device workspace a fit of this shape needs.  Pure host function:
 * usable before any GPU call, e.g. to admit work by HBM footprint.  0 on bad input. */
size_t gap_workspace_bytes(const gap_params *p, int64_t n_configs, int64_t n_atoms, int64_t M);

/* Hand the library a caller-owned device buffer (256-byte aligned) of `bytes`
 * bytes.  The library carves every scratch array from it.  GAP_EINVAL on NULL
 * or misaligned pointers. */
gap_status gap_bind_workspace(gap_handle h, void *dev_ptr, size_t bytes);

/*
 * Build the stacked matrix's blocks (Sec. Theory: K_NM, K_MM, Cholesky; the
 * upper block of A and its lower block L^T).
 *   x_atoms        [n_atoms x d] row-major FP64, atoms of a configuration contiguous
 *   config_offsets [n_configs + 1] int64: configuration A owns atoms
 *                  offsets[A] .. offsets[A+1]-1; offsets[0] = 0, nondecreasing,
 *                  offsets[n_configs] = n_atoms (checked on the device; a violation
 *                  is reported as GAP_EINVAL through the device status)
 *   x_sparse       [M x d] row-major FP64 sparse points
 *   sigma          [n_configs] FP64 standard deviation of each target (> 0)
 * Requires n_configs >= 1, M >= 1, n_atoms >= 1, workspace >= gap_workspace_bytes.
 */
gap_status gap_build_knm(gap_handle h, const double *x_atoms, int64_t n_atoms,
                         const int64_t *config_offsets, int64_t n_configs,
                         const double *x_sparse, int64_t M, const double *sigma);

/* One fit's inputs for gap_build_knm_batch (device pointers, as in gap_build_knm). */
/*
 * Derivative observations (forces, virials; Sec. Theory: their rows of K_NM follow
 * by differentiating the energy expression).  x_grad holds descriptor gradients:
 * row g is d x_i / d r for one position coordinate r, i = grad_atom[g] (an index
 * into x_atoms).  Observation o is a weighted sum over its positions p =
 * obs_offsets[o] .. obs_offsets[o+1]: row o of K is
 *   sum_p pos_weight[p] zeta sigma_w^2 (x_i . x_j)^(zeta - 1) (x_grad[pos_grad[p]] . x_j),
 * i = grad_atom[pos_grad[p]].  A force component F_{k,alpha} = -dE/dr_{k,alpha}
 * takes weight -1 over the gradients with respect to r_{k,alpha}; a virial
 * component -sum_k r_{k,alpha} dE/dr_{k,beta} takes weight -r_{k,alpha} over
 * those with respect to r_{k,beta} (a gradient row may serve several
 * observations).  All arrays are device arrays owned by the caller, kept alive
 * until the build has run.  Checked on the device (GAP_EINVAL in the status,
 * nothing read out of range): obs_offsets[0] == 0, nondecreasing,
 * obs_offsets[n_obs] == n_pos; pos_grad values in [0, n_grad); grad_atom values
 * in [0, n_atoms).
 */
typedef struct gap_deriv_obs {
    const double *x_grad;        /* [n_grad x d] FP64 row-major */
    int64_t n_grad;
    const int64_t *grad_atom;    /* [n_grad] */
    const int64_t *obs_offsets;  /* [n_obs + 1] */
    int64_t n_obs;
    const int64_t *pos_grad;     /* [n_pos] gradient row of each position */
    const double *pos_weight;    /* [n_pos] */
    int64_t n_pos;
} gap_deriv_obs;

/* Workspace bytes for a fit with n_configs energies and n_obs derivative
 * observations over n_pos positions (0 on bad arguments). */
size_t gap_workspace_bytes_obs(const gap_params *p, int64_t n_configs, int64_t n_atoms, int64_t n_obs,
                               int64_t n_pos, int64_t M);

/* gap_build_knm with derivative observations: A's rows are the n_configs
 * energies (as gap_build_knm), then the obs->n_obs derivative observations, then
 * L^T; sigma [n_configs + obs->n_obs] holds every row's standard deviation, and
 * gap_solve then takes y of the same length.  The derivative rows need an extra
 * n_atoms x M FP64 block of the workspace (the powers (x_i . x_j)^(zeta - 1)).
 * GAP_EINVAL with GAP_MIXED_BF16 / GAP_MIXED_FP16 (their low-precision block has
 * energy rows only) or incomplete obs. */
gap_status gap_build_knm_obs(gap_handle h, const double *x_atoms, int64_t n_atoms, const int64_t *config_offsets,
                             int64_t n_configs, const gap_deriv_obs *obs, const double *x_sparse, int64_t M,
                             const double *sigma);

typedef struct gap_batch_fit {
    const double *x_atoms;
    int64_t n_atoms;
    const int64_t *config_offsets;
    int64_t n_configs;
    const double *x_sparse;
    int64_t M;
    const double *sigma;
} gap_batch_fit;

/*
 * The K_NM (Sec. Theory, definition of K_MN) of n fits -- a batch of independent
 * fits such as a hyperparameter sweep -- enqueued on `stream` (a hipStream_t or
 * NULL) as grouped launches: each launch covers the tiles of up to 16 fits in one
 * grid.  Each fit's tile plan and K_NM are what gap_build_knm computes for it
 * (bit for bit).  handles[i] (distinct, each with a bound workspace) takes
 * fits[i]; afterwards each handle needs gap_build_kmm, which runs the rest of its
 * build (K_MM, jitter, Cholesky; the low-precision K_NM in GAP_MIXED_BF16/FP16)
 * on the handle's own stream: the caller orders each handle's stream after
 * `stream` (an event).  GAP_EINVAL / GAP_ENOMEM / GAP_ESTATE as gap_build_knm,
 * before anything is enqueued.  Stage 0 of gap_stage_times is not timed.
 */
gap_status gap_build_knm_batch(gap_handle *handles, int32_t n, const gap_batch_fit *fits, void *stream);

/* The rest of a batched build on the handle's stream (see gap_build_knm_batch).
 * GAP_ESTATE unless the handle's last call was a batched K_NM. */
gap_status gap_build_kmm(gap_handle h);

/*
 * Solve for the weights (Sec. Theory: b = [Sigma^-1/2 y ; 0], Householder QR of
 * [A | b] giving R and Q^T b, back-substitution c = R^-1 (Q^T b)[0:M]).
 *   y      [n_configs] FP64 targets (device); after gap_build_knm_obs
 *          [n_configs + n_obs]: energies, then the derivative observations
 *   c_out  [M] FP64 weights (device)
 *   info   host struct or NULL.  When non-NULL the call waits for the stream and
 *          returns the device status; when NULL it returns after enqueueing.
 * The factorisation overwrites the stacked matrix: call gap_build_knm again
 * before solving with another y.
 */
gap_status gap_solve(gap_handle h, const double *y, double *c_out, gap_solve_info *info);

/*
 * Predict total energies (Eqs. 1-2) of n_configs configurations against the
 * sparse set bound by the last gap_build_knm (or gap_set_model):
 *   y_out[A] = sum_{i in A} sum_j c_j sigma_w^2 (x_i . x_j)^zeta.
 * x_atoms/offsets as in gap_build_knm; c [M] and y_out [n_configs] device FP64.
 * Uses no workspace.  The offsets are checked on the device before any
 * descriptor is read: a configuration whose range is not inside [0, n_atoms),
 * or offsets[0] != 0, or offsets[n_configs] != n_atoms, gives NaN energies for
 * the configurations of its workgroup and GAP_EINVAL in the device status
 * (read by gap_sync): the fit's status word on a fit handle, the first word of
 * a bound workspace on a predict-only handle (none if it has no workspace).
 */
gap_status gap_predict(gap_handle h, const double *x_atoms, int64_t n_atoms,
                       const int64_t *offsets, int64_t n_configs, const double *c, double *y_out);

/* Bind a resident model's sparse set [M x d] (device FP64, caller-owned) for
 * gap_predict without a fit or a workspace (e.g. a served model whose fit has
 * finished and released its workspace).  The handle becomes predict-only: a
 * fit's workspace bound before is no longer used.  A workspace bound after
 * this call (>= 16 bytes) holds the handle's status word, which stays set
 * until the workspace is bound again.  GAP_EINVAL on NULL or M < 1. */
gap_status gap_set_model(gap_handle h, const double *x_sparse, int64_t M);

/* Move the handle to another HIP stream (hipStream_t or NULL) for later calls. */
gap_status gap_set_stream(gap_handle h, void *stream);

/* Wait for the handle's stream; fill info (nullable) and return the device status. */
gap_status gap_sync(gap_handle h, gap_solve_info *info);

/* Where the stage outputs live in the workspace (after gap_build_knm). */
gap_status gap_layout(gap_handle h, gap_layout_info *out);

/* Per-stage milliseconds of the last build/solve when GAP_FLAG_TIMING is set:
 * [0] K_NM kernel, [1] K_MM kernel, [2] Cholesky, [3] b assembly,
 * [4] Householder QR incl. Q^T b, [5] back-substitution, [6] refinement,
 * [7] low-precision K_NM (rounding the descriptors and the BF16/FP16 kernel),
 * [8] solution diagnostics (grad_rel, and est_err when requested),
 * [9] derivative observation rows (gap_build_knm_obs).
 * Waits for the stream.  n = number of floats in ms (up to 10). */
gap_status gap_stage_times(gap_handle h, float *ms, int n);

/* Launch-shape and method knobs an autotuner may set per handle (0 = library default).
 *   qr_split_wgs  target number of workgroups of the QR's split-K products
 *                 Y^T C (sets the row-chunk height); 256 .. 65536.
 *   qr_panel      panel factorisation of the Householder QR: 0 = shifted
 *                 CholeskyQR3 (streams the panel; default), 1 = TSQR over a
 *                 4-ary tree of 256-row tiles.  Both end in the same
 *                 reconstructed Householder representation.
 *   qr_lookahead  0 = automatic (look-ahead from M >= 2048 on), 1 = off (the
 *                 whole QR on the handle's stream), 2 = on.  Look-ahead: the
 *                 trailing update of each 128-column block runs on a second
 *                 stream the handle owns while the handle's stream updates and
 *                 factors the next block.  The two schedules sum the split-K
 *                 partials of the next block's update over different row chunks,
 *                 so they agree to rounding; each one is deterministic.
 *   qr_free_cus   look-ahead only: 1 .. 128 CUs kept free of the trailing-update
 *                 stream (a HIP CU mask) for the next block's panel chain on the
 *                 handle's stream; 0 = no mask (default).  At N = 1e5, M = 1e4
 *                 on MI355X, 32 is best in both precisions.  A masked stream is a blocking one: it
 *                 orders itself with the legacy default stream, so use it for a
 *                 handle on a stream of its own in a process that keeps work off
 *                 the legacy stream meanwhile; a captured graph does not keep
 *                 the mask.  Takes effect at the next gap_build_knm (which
 *                 replaces the stream after its last work); results are
 *                 unchanged.
 *   knm_bn        K_NM column tile: 64 sparse points (0 or 64, default) or 32.
 *                 Each entry's arithmetic does not depend on it: results are
 *                 bitwise unchanged. */
typedef struct gap_tuning {
    int32_t qr_split_wgs;
    int32_t qr_panel;
    int32_t qr_lookahead;
    int32_t qr_free_cus;
    int32_t knm_bn;
    int32_t reserved[3];
} gap_tuning;

/* Set the handle's launch-shape knobs (host-only; affects later calls).  GAP_EINVAL on
 * out-of-range values. */
gap_status gap_set_tuning(gap_handle h, const gap_tuning *t);

/*
 * Allocation-free fit, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): gap_build_knm + gap_solve of one fit with the same arguments and
 * the same kernels, but with the library's scratch in a static device array
 * of GAP_STATIC_SCRATCH_BYTES per GPU (allocated when the library's code is
 * loaded on that GPU and held until the process ends) instead of a bound
 * workspace.  No handle is kept: the call allocates no device or host memory
 * and creates no stream or event (the QR runs without look-ahead, and
 * GAP_FLAG_TIMING is rejected).  Inputs and outputs are the caller's device
 * arrays, as in gap_build_knm / gap_solve; `info` as in gap_solve (non-NULL:
 * wait and return the device status; NULL: return after enqueueing).
 * GAP_ENOMEM when gap_workspace_bytes() of this shape exceeds
 * GAP_STATIC_SCRATCH_BYTES.  Every call on one GPU uses that GPU's one
 * array, which keeps the last call's contents: calls that overlap on one GPU
 * (other host threads, or other streams before the previous call's work has
 * finished) race and give wrong results.  Each call clears the counters and
 * flags it relies on with kernels (no memset nodes), so it may be captured.
 */
#define GAP_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
gap_status gap_fit_static(const gap_params *p, void *stream, const double *x_atoms, int64_t n_atoms,
                          const int64_t *config_offsets, int64_t n_configs, const double *x_sparse, int64_t M,
                          const double *sigma, const double *y, double *c_out, gap_solve_info *info);
/* GAP_STATIC_SCRATCH_BYTES (for callers that load the library dynamically). */
size_t gap_static_scratch_bytes(void);

/*
 * CUR sparse-point selection (Sec. Implementation: the sparse points are chosen
 * from the descriptor rows by CUR-based methods, after Mahoney & Drineas 2009).
 * For the n_rows x d matrix X of descriptor rows (device FP64, row-major), the
 * leverage of row i over the row space of X is
 *   lev_i = x_i^T (X^T X)^-1 x_i   (the hat matrix's diagonal; sum_i lev_i = d).
 * exp_draws == NULL: the M rows of largest leverage.  Otherwise exp_draws[i] is
 * an Exp(1) variate per row, drawn by the caller, and the M rows of smallest
 * key exp_draws[i] / lev_i are taken: a sample without replacement with
 * probabilities proportional to the leverage (Efraimidis & Spirakis).  Keys
 * are formed in FP64; equal keys are taken in row order; rows with lev_i = 0
 * get an infinite key.
 *   selected      [M] device int64: the selected row indices, ascending.
 *   leverage      [n_rows] device FP64 or NULL: lev_i.
 *   workspace     device scratch of gap_cur_workspace_bytes(n_rows, d) bytes,
 *                 caller-owned; its first 64 bytes hold the device status.
 * Enqueued on `stream`.  wait != 0: synchronise the stream and return the
 * device status (GAP_ENOTPD when a pivot of the Cholesky factorisation of
 * X^T X is not positive, e.g. X has a zero column: the output is then
 * meaningless; a rank deficiency that rounding hides is not detected, and the
 * leverages carry an error of about kappa(X)^2 u); wait == 0: return GAP_OK
 * after enqueueing.  GAP_EINVAL on NULL x/selected/workspace, n_rows < d,
 * d < 1 or d > 4096, M < 1 or M > n_rows; GAP_ENOMEM when workspace_bytes is
 * too small.  Inputs are not modified.
 */
size_t gap_cur_workspace_bytes(int64_t n_rows, int32_t d);
gap_status gap_cur_select(const double *x, int64_t n_rows, int32_t d, const double *exp_draws, int64_t M,
                          int64_t *selected, double *leverage, void *workspace, size_t workspace_bytes,
                          void *stream, int32_t wait);

/* Human-readable name of a status code (static string). */
const char *gap_status_string(gap_status s);

/* Release the handle (host memory and events).  The workspace stays the caller's. */
gap_status gap_destroy(gap_handle h);

#ifdef __cplusplus
}
#endif

#endif /* GAP_H */
