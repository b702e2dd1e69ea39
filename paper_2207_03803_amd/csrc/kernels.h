// Internal kernel interfaces of the GAP fit library.  Every launcher enqueues
// on the given stream and returns the launch error (hipSuccess when none).
#pragma once

#include "common.h"
#include "knm.h"

namespace gap {

// ------------------------------------------------------------------- Cholesky
constexpr int CHOL_NB = 64;
// In-place upper Cholesky K = U^T U of the n x n matrix at U (column-major,
// leading dimension ld; only the upper triangle is read, U written there, the
// strictly lower part of each diagonal block zeroed).  First non-positive
// pivot -> status DST_ENOTPD.
hipError_t launch_potrf_upper(double *U, int64_t ld, int64_t n, int32_t *status, hipStream_t s);

// ----------------------------------------------------- CUR sparse-point selection
// Leverages of the n rows of X [n x d] (row-major FP64) over its row space, keys
// draws[i] / lev[i] (1 / lev[i] when draws is null), and the M rows of smallest
// key in ascending order into out.  The device status (DST_ENOTPD when X^T X is
// not positive definite) is the first int32 of cur_status_offset() in the
// workspace of cur_workspace_bytes(n, d) bytes.
struct CurLaunch {
    const double *x;
    int64_t n;
    int d;
    const double *draws;  // [n] or null
    int64_t M;
    int64_t *out;         // [M]
    double *lev_out;      // [n] or null
    void *workspace;
};
size_t cur_workspace_bytes(int64_t n, int d);
size_t cur_status_offset();
int cur_max_d();
hipError_t launch_cur_select(const CurLaunch &c, hipStream_t s);

// ------------------------------------------------------------ Householder QR
constexpr int QR_NB = 64;        // panel width
constexpr int TS_ROWS = 256;     // rows of one TSQR tile
constexpr int TS_FAN = 4;        // children per TSQR tree node
constexpr int TS_MAX_LEVELS = 16;

// TSQR tree storage for panels of up to m rows.  Level 0 has ceil(m/256)
// nodes, level l+1 has ceil(n_l / 4).  Every node owns a 256 x 64 tile
// (column-major inside the tile), 64 reflector weights and (levels >= 1) a
// 256 x 64 block of the explicit Q.
struct TsqrTree {
    int levels = 0;
    int64_t nodes[TS_MAX_LEVELS] = {};
    int64_t tile_off[TS_MAX_LEVELS] = {};  // offsets in doubles into tiles / X
    int64_t tau_off[TS_MAX_LEVELS] = {};   // offsets in doubles into tau
    int64_t tiles_doubles = 0, tau_doubles = 0;
};
TsqrTree tsqr_tree(int64_t m);

struct QrWork {
    double *A;        // column-major [lda x ncols]: factor columns 0..n-1, apply to n..ncols-1
    float *A32;       // when non-null: factor this FP32 copy instead (same layout); A is not touched
    int64_t lda, m, n, ncols;
    int64_t tri0;     // rows [tri0, m) are upper triangular from column 0 (row tri0 + i is zero in the
                      // columns before i) and are skipped until the factorisation reaches them; 0: none
    int64_t ldw;      // leading dimension of W (ncols rounded up to 64)
    double *tau;      // [n]
    double *wpart;    // [max_chunks * 4 QR_NB * wp_ld] split-K partials of Y^T C
    int64_t wp_ld;    // row stride of the partials (>= the widest column range updated)
    double *T;        // [16 QR_NB^2] compact-WY data of the current four-panel block (T_a, T_b, G, H)
    double *T2;       // second T buffer (look-ahead: the side stream reads one while the next is formed)
    double *wpart_s;  // [qr_max_chunks_s() * 4 QR_NB * 2 QR_NB] partials of the main stream's small updates
    double *W_s;      // [4 QR_NB * 4 QR_NB] W of the main stream's small updates (ld 2 or 4 QR_NB)
    float *W32_s;     // FP32 version
    double *Tin;      // [2 * QR_NB * QR_NB] T of the block's two panels (row-major, ld QR_NB)
    double *U;        // [QR_NB * QR_NB] LU factor of (Q - S) of the current panel
    double *W;        // [4 QR_NB * ldw] T^T Y^T C, row-major by block column
    float *W32;       // same for the FP32 factorisation
    double *ts_tiles; // TsqrTree::tiles_doubles
    double *ts_X;     // TsqrTree::tiles_doubles
    double *ts_tau;   // TsqrTree::tau_doubles
    TsqrTree tree;    // sized for m rows
    int64_t max_chunks;
    int32_t split_wgs;  // target workgroups of the split-K products (0 = default)
    int32_t panel;      // panel factorisation: 0 = shifted CholeskyQR3, 1 = TSQR
    double *cq_S;       // CholeskyQR: FP64 scratch panel [QR_NB x cq_ld] (column-major)
    int64_t cq_ld;      // >= m
    double *cq_part;    // [CQ_MAX_CHUNKS * QR_NB * QR_NB] partial Gram matrices
    double *cq_G;       // [4 * QR_NB * QR_NB] four partial sums of the Gram matrix
    double *cq_R;       // [4 * QR_NB * QR_NB] R1, R2, R2 R1, U R3 (row-major)
    int32_t *status;
};
constexpr int64_t CQ_MAX_CHUNKS = 256;
// Shifted CholeskyQR3 panel + Householder reconstruction (same outputs as the TSQR panel).
void cqr_panel_f64(const QrWork &w, int64_t j0, int pw, double *Tout, hipStream_t s);
void cqr_panel_f32(const QrWork &w, int64_t j0, int pw, double *Tout, hipStream_t s);
int64_t qr_max_chunks();
int64_t qr_max_chunks_s();
// Look-ahead schedule: the trailing update of block k runs on `side` while
// `s` updates block k+1's columns and factors them.  Null: one stream.
struct QrAsync {
    hipStream_t side;
    hipEvent_t fork, t_ready, bulk[2], join;
};
hipError_t launch_geqrf(const QrWork &w, hipStream_t s, const QrAsync *la);

// -------------------------------------------------------- triangular solve
// Flags of the one-launch blocked substitution: sync.flags holds
// trsv_sync_ints(n) int32 (zero before the first solve; each solve leaves them
// zero), sync.counter one unsigned (zero), sync.status the device status word.
struct TrsvSync {
    int32_t *flags;
    unsigned *counter;
    int32_t *status;
};
int64_t trsv_sync_ints(int64_t n);
// Solve R c = rhs for the n x n upper triangle of R (column-major, ld); then
// check c is finite (DST_ENONFINITE otherwise).
hipError_t launch_trsv_upper(const double *R, int64_t ld, int64_t n, const double *rhs, double *c,
                             const TrsvSync &sync, hipStream_t s);
// Same with R stored in FP32 (FP64 arithmetic).
hipError_t launch_trsv_upper_f32(const float *R, int64_t ld, int64_t n, const double *rhs, double *x,
                                 const TrsvSync &sync, const int32_t *skip, hipStream_t s);
// FP64 R without the finiteness check, and R^T x = rhs with the FP64 R.
hipError_t launch_trsv_upper_nc(const double *R, int64_t ld, int64_t n, const double *rhs, double *x,
                                const TrsvSync &sync, hipStream_t s);
hipError_t launch_trsv_upper_t(const double *R, int64_t ld, int64_t n, const double *rhs, double *x,
                               const TrsvSync &sync, hipStream_t s);
// Solve R^T x = rhs (forward substitution) for the FP32-stored upper R.
hipError_t launch_trsv_upper_t_f32(const float *R, int64_t ld, int64_t n, const double *rhs, double *x,
                                   const TrsvSync &sync, const int32_t *skip, hipStream_t s);
hipError_t launch_copy_f32_f64(const float *src, double *dst, int64_t n, hipStream_t s);
hipError_t launch_sumsq(const double *x, int64_t n, double *out, double *part, unsigned *counter,
                        hipStream_t s);

// ------------------------------------------------------ mixed-precision refinement
struct RefineWork {
    const double *A;     // FP64 [A | b], column-major lda; b is column n
    int64_t lda, m, n;
    const float *R32;    // FP32 factor (upper triangle of the first n rows), same lda
    double *c;           // [n] solution, refined in place
    double *r;           // [m] residual
    double *s, *z, *dc;  // [n] work
    double *p;           // [n] CGLS search direction
    double *q;           // [m] A p
    double *part;        // [8 * m] column-chunk partials of A c (A p)
    double *rnorm_part;  // [ceil(m / 256)] partial ||r||^2 (||q||^2)
    int32_t *done;       // convergence flag
    int32_t *iters;      // [0] iterations done, [1] of them CGLS steps
    int32_t *mode;       // refinement stage: CSNE, CGLS start, CGLS step
    double *stats;       // [0] ||r||^2, [1] last step / ||c||, [2] CGLS alpha, [3] CGLS gamma
    double tol;
    int32_t *status;
    TrsvSync sync;       // flags of the triangular solves
};
hipError_t launch_convert_f64_f32(const double *a, float *b, int64_t n, hipStream_t s);
// Rows [r0, r1) of columns [c0, c1) of a column-major FP64 matrix into its FP32 copy (same ld).
hipError_t launch_convert_block_f64_f32(const double *a, float *b, int64_t ld, int64_t r0, int64_t r1, int64_t c0,
                                        int64_t c1, hipStream_t s);
hipError_t launch_refine(const RefineWork &w, int max_iters, hipStream_t s);

// ---------------------------------------------------------------- diagnostics
// Normal-equation residual eta of the returned weights and (iters > 0) the
// error estimate u (kappa + kappa^2 ||r|| / (||A||_2 ||c||)) from power and
// inverse iteration on R.  out[0] = eta, out[1] = estimate (-1 without one),
// out[2] = kappa estimate.
struct DiagWork {
    int64_t n, ld;
    double *part;        // [8 * n] column-chunk partials of R x
    double *partR;       // [n] column sums of R^2
    double *t, *g;       // [n]: (Q^T b)[0:n] - R c (FP64), A^T r
    double *x, *y, *z;   // [n]: iteration vectors
    double *sc;          // [4] scalars
    double *sum_part;    // [256] partials of launch_sumsq
    unsigned *counter;   // its arrival counter (zero)
    const double *tail2; // FP64: minimum loss ||(Q^T b)[n:]||^2 (device scalar)
    int iters;           // steps of each iteration (0: no estimate)
    TrsvSync sync;
};
hipError_t launch_diag_fp64(const DiagWork &d, const double *R, const double *qtb, const double *c, double *out,
                            hipStream_t s);
// Mixed precision: d.g already holds A^T r at c (FP64 A); r2 = device ||r||^2;
// bcol = the FP64 b (m entries); R32 = the FP32 factor.
hipError_t launch_diag_mixed(const DiagWork &d, const float *R32, const double *bcol, int64_t m, const double *r2,
                             const double *c, double *out, hipStream_t s);

// ---------------------------------------------------------------- utilities
// b = [y / sigma ; 0] into column `col` of the column-major A (lda rows).
hipError_t launch_assemble_b(const double *y, const double *sigma, int64_t N, double *bcol,
                             int64_t lda, hipStream_t s);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);
// Zero rows [r0, r1) of columns [c0, c1) of a column-major matrix.
hipError_t launch_zero_block(double *A, int64_t lda, int64_t r0, int64_t r1, int64_t c0, int64_t c1,
                             hipStream_t s);
hipError_t launch_check_finite(const double *x, int64_t n, int32_t *status, hipStream_t s);

}  // namespace gap
