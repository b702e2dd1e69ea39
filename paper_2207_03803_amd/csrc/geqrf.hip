// Blocked Householder QR of the augmented stacked matrix [A | b] in FP64
// (Sec. Implementation: the factorisation leaves R in the upper triangle and
// the Householder vectors below it with their weights tau; Q^T b comes from
// carrying b along as an extra column, which is what applying the stored
// reflectors to b computes).
//
// Each 64-column panel is factored by shifted CholeskyQR3 (cqr.hip) or, as
// selected per handle, as a tall-skinny QR (TSQR) over a 4-ary tree of
// 256-row tiles with its explicit Q formed top-down; in both cases the
// Householder vectors Y and the compact-WY factor T recovered from that Q by
// an LU factorisation of Q - S with the sign matrix S chosen to keep every
// pivot at least 1 in magnitude (Ballard, Demmel, Grigori, Jacquelin, Knight,
// Nguyen 2015, "Reconstructing Householder vectors from tall-skinny QR").  The
// result is the LAPACK-style representation H = I - Y T Y^T with Y unit lower
// trapezoidal, R = S R_tsqr, tau_i = T_ii.  The trailing columns (b included)
// are then updated on MFMA: P = Y^T C (split over row chunks), W = T^T P,
// C -= Y W.
//
// Reflector convention inside the tiles: H = I - tau v v^T, v(0) = 1,
// beta = -sign(alpha) ||(alpha, x)||, tau = (beta - alpha)/beta,
// v(1:) = x / (alpha - beta); tau = 0 when x is exactly zero.
#include "kernels.h"

namespace gap {

constexpr int NB = QR_NB;
constexpr int TR = TS_ROWS;
constexpr int TILE = TR * NB;  // doubles per tile
constexpr int NPART = 8;           // threads per tile column
constexpr int TS_NT = NB * NPART;  // threads of the TSQR kernels
constexpr int SLOTS = TR / NPART;  // rows held per thread (row = NPART * slot + part)
constexpr int64_t MAX_CHUNKS = 32;     // row chunks of the split-K products into the bulk buffer
constexpr int64_t MAX_CHUNKS_S = 256;  // into the small buffer at 2 QR_NB columns (half that at 4 QR_NB)

int64_t qr_max_chunks() { return MAX_CHUNKS; }
int64_t qr_max_chunks_s() { return MAX_CHUNKS_S; }

TsqrTree tsqr_tree(int64_t m)
{
    TsqrTree t;
    int64_t n = (m + TR - 1) / TR;
    int64_t toff = 0, aoff = 0;
    for (int l = 0; l < TS_MAX_LEVELS; ++l) {
        t.nodes[l] = n;
        t.tile_off[l] = toff;
        t.tau_off[l] = aoff;
        toff += n * TILE;
        aoff += n * NB;
        t.levels = l + 1;
        if (n <= 1)
            break;
        n = (n + TS_FAN - 1) / TS_FAN;
    }
    t.tiles_doubles = toff;
    t.tau_doubles = aoff;
    return t;
}

// Node counts for a panel of mk rows (never more than the tree was sized for).
struct PanelTree {
    int levels;
    int64_t nodes[TS_MAX_LEVELS];
};

static PanelTree panel_tree(int64_t mk)
{
    PanelTree p{};
    int64_t n = (mk + TR - 1) / TR;
    for (int l = 0; l < TS_MAX_LEVELS; ++l) {
        p.nodes[l] = n;
        p.levels = l + 1;
        if (n <= 1)
            break;
        n = (n + TS_FAN - 1) / TS_FAN;
    }
    return p;
}

// Rows [lo, hi) of level-0 tile i out of n0 (balanced split of mk rows).
DEV void leaf_rows(int64_t i, int64_t n0, int64_t mk, int64_t &lo, int64_t &hi)
{
    lo = (i * mk) / n0;
    hi = ((i + 1) * mk) / n0;
}

// The matrix being factored: FP64 storage (w.A) or FP32 storage (w.A32).
template <class T>
DEV T *qmat(const QrWork &w);
template <>
DEV double *qmat<double>(const QrWork &w) { return w.A; }
template <>
DEV float *qmat<float>(const QrWork &w) { return w.A32; }

// Sum over the NPART consecutive lanes that hold one column (deterministic).
DEV double col_sum(double v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Householder QR of one 256 x pw tile held in registers.  Thread t owns
// column q = t / 8 and the rows r = 8 * slot + (t % 8).  Level 0 reads rows
// of the panel; level l >= 1 stacks the R factors of up to 4 children.  The
// factored tile (R above the diagonal, v below) and tau go to the tree.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(TS_NT) void tsqr_factor_kernel(QrWork w, int64_t j0, int pw, int level,
                                                          int64_t n_level, int64_t n_prev, int64_t mk)
{
    __shared__ double vbuf[2][TR];
    __shared__ double taus[NB];
    const int t = threadIdx.x, q = t / NPART, part = t % NPART;
    const int64_t node = blockIdx.x;
    double x[SLOTS];
    if (level == 0) {
        int64_t lo, hi;
        leaf_rows(node, n_level, mk, lo, hi);
        const T *col = qmat<T>(w) + (j0 + q) * w.lda + j0 + lo;
        const int64_t nr = hi - lo;
#pragma unroll
        for (int i = 0; i < SLOTS; ++i) {
            const int r = NPART * i + part;
            x[i] = (q < pw && r < nr) ? (double)col[r] : 0.0;
        }
    } else {
        const double *prev = w.ts_tiles + w.tree.tile_off[level - 1];
        const int64_t c0 = node * TS_FAN;
        const int64_t nc = (n_prev - c0) < TS_FAN ? (n_prev - c0) : TS_FAN;
#pragma unroll
        for (int i = 0; i < SLOTS; ++i) {
            const int r = NPART * i + part;
            const int k = r / pw, rr = r % pw;
            x[i] = (q < pw && k < nc && rr <= q) ? prev[(c0 + k) * TILE + q * TR + rr] : 0.0;
        }
    }
    for (int j = 0; j < pw; ++j) {
        double *v = vbuf[j & 1];
        if (q == j) {
            double s = 0.0, a = 0.0;
#pragma unroll
            for (int i = 0; i < SLOTS; ++i) {
                const int r = NPART * i + part;
                if (r > j)
                    s += x[i] * x[i];
                if (r == j)
                    a = x[i];
            }
            s = col_sum(s);
            a = col_sum(a);  // one lane holds alpha, the others 0
            double tau = 0.0, scale = 0.0, beta = a;
            if (s != 0.0) {
                const double norm = sqrt(a * a + s);
                beta = (a >= 0.0) ? -norm : norm;
                tau = (beta - a) / beta;
                scale = 1.0 / (a - beta);
            }
#pragma unroll
            for (int i = 0; i < SLOTS; ++i) {
                const int r = NPART * i + part;
                if (r == j)
                    x[i] = beta;
                else if (r > j)
                    x[i] *= scale == 0.0 ? 1.0 : scale;
                v[r] = (r == j) ? 1.0 : (r > j ? x[i] : 0.0);
            }
            if (part == 0)
                taus[j] = tau;
        }
        __syncthreads();
        const double tau = taus[j];
        if (q > j && q < pw && tau != 0.0) {
            double d = 0.0;
#pragma unroll
            for (int i = 0; i < SLOTS; ++i)
                d += v[NPART * i + part] * x[i];
            d = col_sum(d) * tau;
#pragma unroll
            for (int i = 0; i < SLOTS; ++i)
                x[i] -= d * v[NPART * i + part];
        }
    }
    double *out = w.ts_tiles + w.tree.tile_off[level] + node * TILE + q * TR;
#pragma unroll
    for (int i = 0; i < SLOTS; ++i)
        out[NPART * i + part] = x[i];
    if (part == 0)
        w.ts_tau[w.tree.tau_off[level] + node * NB + q] = (q < pw) ? taus[q] : 0.0;
}

// ---------------------------------------------------------------------------
// Explicit Q, top-down: X_node = H_0 H_1 ... H_{pw-1} [S ; 0] where S is the
// node's pw x pw slice of its parent's X (the identity at the root).  Level 0
// writes its X into the panel's rows of A.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(TS_NT) void tsqr_formq_kernel(QrWork w, int64_t j0, int pw, int level,
                                                         int64_t n_level, int is_root, int64_t mk)
{
    __shared__ double V[NB * (TR + 1)];
    __shared__ double taus[NB];
    const int t = threadIdx.x, q = t / NPART, part = t % NPART;
    const int64_t node = blockIdx.x;
    const double *tile = w.ts_tiles + w.tree.tile_off[level] + node * TILE;
    for (int idx = t; idx < TILE; idx += TS_NT) {
        const int c = idx / TR, r = idx % TR;
        V[c * (TR + 1) + r] = tile[idx];
    }
    if (t < NB)
        taus[t] = w.ts_tau[w.tree.tau_off[level] + node * NB + t];
    double x[SLOTS];
    if (is_root) {
#pragma unroll
        for (int i = 0; i < SLOTS; ++i) {
            const int r = NPART * i + part;
            x[i] = (r == q && q < pw) ? 1.0 : 0.0;
        }
    } else {
        const int64_t parent = node / TS_FAN, pos = node % TS_FAN;
        const double *px = w.ts_X + w.tree.tile_off[level + 1] + parent * TILE + q * TR + pos * pw;
#pragma unroll
        for (int i = 0; i < SLOTS; ++i) {
            const int r = NPART * i + part;
            x[i] = (q < pw && r < pw) ? px[r] : 0.0;
        }
    }
    __syncthreads();
    if (q < pw) {
        for (int j = pw - 1; j >= 0; --j) {
            const double tau = taus[j];
            if (tau == 0.0)
                continue;
            const double *vc = V + j * (TR + 1);
            double d = 0.0;
#pragma unroll
            for (int i = 0; i < SLOTS; ++i) {
                const int r = NPART * i + part;
                const double vr = (r > j) ? vc[r] : (r == j ? 1.0 : 0.0);
                d += vr * x[i];
            }
            d = col_sum(d) * tau;
#pragma unroll
            for (int i = 0; i < SLOTS; ++i) {
                const int r = NPART * i + part;
                const double vr = (r > j) ? vc[r] : (r == j ? 1.0 : 0.0);
                x[i] -= d * vr;
            }
        }
    }
    if (level == 0) {
        int64_t lo, hi;
        leaf_rows(node, n_level, mk, lo, hi);
        if (q < pw) {
            T *col = qmat<T>(w) + (j0 + q) * w.lda + j0 + lo;
            const int64_t nr = hi - lo;
#pragma unroll
            for (int i = 0; i < SLOTS; ++i) {
                const int r = NPART * i + part;
                if (r < nr)
                    col[r] = (T)x[i];
            }
        }
    } else {
        double *out = w.ts_X + w.tree.tile_off[level] + node * TILE + q * TR;
#pragma unroll
        for (int i = 0; i < SLOTS; ++i)
            out[NPART * i + part] = x[i];
    }
}

// ---------------------------------------------------------------------------
// Reconstruction, top block (one workgroup): LU of Q1 - S with s_k =
// -sign(pivot) (sign(0) = +1), giving U and the unit lower Y1; then
// T = -U S Y1^-T, R = S R_root; writes R above and Y1 below the diagonal of
// the panel's top block, tau = diag(T), and U for the row solve below.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void tsqr_lu_kernel(QrWork w, int64_t j0, int pw, int root_level, double *Tout)
{
    __shared__ double B[NB][NB + 1];
    __shared__ double Z[NB][NB + 1];
    __shared__ double sg[NB];
    const int t = threadIdx.x;
    for (int idx = t; idx < pw * pw; idx += 256) {
        const int r = idx % pw, c = idx / pw;
        B[r][c] = (double)qmat<T>(w)[(j0 + c) * w.lda + j0 + r];
    }
    __syncthreads();
    for (int k = 0; k < pw; ++k) {
        if (t == 0) {
            const double d = B[k][k];
            const double s = (d >= 0.0) ? -1.0 : 1.0;
            B[k][k] = d - s;
            sg[k] = s;
        }
        __syncthreads();
        const double piv = B[k][k];
        for (int i = k + 1 + t; i < pw; i += 256)
            B[i][k] /= piv;
        __syncthreads();
        const int wdt = pw - k - 1;
        for (int idx = t; idx < wdt * wdt; idx += 256) {
            const int i = k + 1 + idx % wdt, c = k + 1 + idx / wdt;
            B[i][c] -= B[i][k] * B[k][c];
        }
        __syncthreads();
    }
    // Z = Y1^-T (unit upper): column c by back-substitution, one thread per column
    if (t < pw) {
        const int c = t;
        for (int r = pw - 1; r >= 0; --r) {
            double v = (r == c) ? 1.0 : 0.0;
            if (r < c)
                for (int p = r + 1; p <= c; ++p)
                    v -= B[p][r] * Z[p][c];
            Z[r][c] = (r <= c) ? v : 0.0;
        }
    }
    __syncthreads();
    const double *root = w.ts_tiles + w.tree.tile_off[root_level];  // node 0
    for (int idx = t; idx < NB * NB; idx += 256) {
        const int r = idx / NB, c = idx % NB;
        double tv = 0.0;
        if (r < pw && c < pw && r <= c) {
            for (int p = r; p <= c; ++p)
                tv -= B[r][p] * sg[p] * Z[p][c];
        }
        Tout[idx] = tv;
        w.U[idx] = (r < pw && c < pw && r <= c) ? B[r][c] : 0.0;
        if (r < pw && c < pw) {
            double out;
            if (r <= c)
                out = sg[r] * root[c * TR + r];
            else
                out = B[r][c];
            qmat<T>(w)[(j0 + c) * w.lda + j0 + r] = (T)out;
        }
        if (r == c && r < pw)
            w.tau[j0 + r] = tv;
    }
}

// Rows below the top block: Y = Q U^-1 (one row per thread).
template <class T>
__global__ __launch_bounds__(256) void tsqr_trsm_kernel(QrWork w, int64_t j0, int pw)
{
    __shared__ double U[NB][NB + 1];
    for (int idx = threadIdx.x; idx < NB * NB; idx += 256)
        U[idx / NB][idx % NB] = w.U[idx];
    __syncthreads();
    const int64_t r = j0 + pw + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= w.m)
        return;
    double y[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c)
        y[c] = (c < pw) ? (double)qmat<T>(w)[(j0 + c) * w.lda + r] : 0.0;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        if (c < pw) {
            double v = y[c];
#pragma unroll
            for (int i = 0; i < c; ++i)
                v -= y[i] * U[i][c];
            y[c] = v / U[c][c];
        }
    }
#pragma unroll
    for (int c = 0; c < NB; ++c)
        if (c < pw)
            qmat<T>(w)[(j0 + c) * w.lda + r] = (T)y[c];
}

// Householder vectors of the column block at (j0, j0), pw <= 2 * QR_NB wide:
// unit lower trapezoidal.
template <class T>
DEV T ypanel(const T *A, int64_t lda, int64_t m, int64_t j0, int pw, int64_t r, int p)
{
    if (p >= pw || r >= m)
        return T(0);
    const int64_t d = r - (j0 + p);
    if (d < 0)
        return T(0);
    if (d == 0)
        return T(1);
    return A[(j0 + p) * lda + r];
}

// Tile of a trailing-update product: logical tiles are numbered row block by
// row block (the column tiles of one row block consecutive), and consecutive
// logical tiles run on the same XCD, so that the row block's Y tile stays in
// that XCD's L2 while its column tiles go by.
DEV bool update_tile(int64_t n_rb, int64_t n_cb, int64_t &rb, int64_t &cb)
{
    const int64_t total = n_rb * n_cb;
    const int64_t lw = xcd_remap(blockIdx.x, (total + 7) & ~int64_t(7));
    if (lw >= total)
        return false;
    rb = lw / n_cb;
    cb = lw % n_cb;
    return true;
}

// Row-block split of a trailing update: PART 0 every row block, 1 the interior
// ones (n_head .. n_rb - 2: full rows, below Y's unit triangle, loaded without
// checks), 2 the edge ones (the n_head row blocks that meet Y's triangle, and
// n_rb - 1).
template <int PART>
DEV bool update_tile_part(int64_t n_rb, int64_t n_cb, int n_head, int64_t &rb, int64_t &cb)
{
    if constexpr (PART == 1) {
        if (!update_tile(n_rb - n_head - 1, n_cb, rb, cb))
            return false;
        rb += n_head;
    } else if constexpr (PART == 2) {
        if (!update_tile(n_head + 1, n_cb, rb, cb))
            return false;
        if (rb == n_head)
            rb = n_rb - 1;
    } else {
        if (!update_tile(n_rb, n_cb, rb, cb))
            return false;
    }
    return true;
}

constexpr int OB = 2 * NB;                 // a TSQR panel pair (one factor_block)
constexpr int OB2 = 2 * OB;                // outer block of the trailing update: two panel pairs
// Both on 16x16x4 MFMA.  The update's 64 x 128 tiles with 8-deep slices (122
// VGPRs, up to four waves per SIMD) measured 1-2 % faster than 128 x 128 x 16
// tiles at two waves per SIMD.
using WS = TileShape<OB, 128, 16, 2, 2, true>;  // P = Y^T C over a row chunk
using US = TileShape<64, 128, 8, 2, 2, true>;   // C^T -= W^T Y^T (rows of C along the MFMA N axis)

// P[ch][p][q] = sum over the chunk's rows r of Y[r][p] C[r][q].  Y is the
// block at (j0, j0) of width pw; C is either columns c0 .. c0+nt of A
// (ymode = 0) or the unit lower trapezoidal block at (c0, c0) of width nt
// (ymode = 1, used for Y_A^T Y_B).  Rows r0 .. m.
__global__ __launch_bounds__(256, 2) void qr_wpart_kernel(QrWork w, int64_t j0, int pw, int64_t c0, int64_t nt,
                                                          int ymode, int64_t r0, int64_t chunk)
{
    __shared__ double lds[2 * WS::STAGE];
    // blockIdx.z: which 128-column half of a block of up to 256 (rows OB z .. of P)
    const int prow0 = OB * (int)blockIdx.z;
    j0 += prow0;
    pw = (pw - prow0) < OB ? (pw - prow0) : OB;
    if (pw <= 0)
        return;
    const int64_t ch = blockIdx.y;
    const int64_t q0 = (int64_t)blockIdx.x * WS::BN;
    const int64_t rlo = r0 + ch * chunk;
    int64_t rhi = rlo + chunk;
    if (rhi > w.m)
        rhi = w.m;
    if (rlo >= rhi)
        return;
    d4 acc[WS::FM][WS::FN];
    zero_acc<WS>(acc);
    const double *A = w.A;
    const int64_t lda = w.lda, m = w.m;
    const bool masked = rlo < j0 + pw;  // the chunk meets Y's unit upper triangle
    constexpr int VA = WS::BM * WS::BK / WS::NT, VB = WS::BN * WS::BK / WS::NT;
    auto fa = [&](int p, int64_t k, double (&v)[VA]) {
        const int64_t r = rlo + k;
        if (p >= pw) {
#pragma unroll
            for (int e = 0; e < VA; ++e)
                v[e] = 0.0;
        } else if (!masked && r + VA <= rhi) {
            load_run(A + (j0 + p) * lda + r, v);
        } else {
#pragma unroll
            for (int e = 0; e < VA; ++e)
                v[e] = (r + e < rhi) ? ypanel(A, lda, m, j0, pw, r + e, p) : 0.0;
        }
    };
    auto fb = [&](int qi, int64_t k, double (&v)[VB]) {
        const int64_t r = rlo + k, q = q0 + qi;
        if (q >= nt) {
#pragma unroll
            for (int e = 0; e < VB; ++e)
                v[e] = 0.0;
        } else if (ymode) {
#pragma unroll
            for (int e = 0; e < VB; ++e)
                v[e] = (r + e < rhi) ? ypanel(A, lda, m, c0, (int)nt, r + e, (int)q) : 0.0;
        } else {
            const double *col = A + (c0 + q) * lda + r;
            if (r + VB <= rhi) {
                load_run(col, v);
            } else {
#pragma unroll
                for (int e = 0; e < VB; ++e)
                    v[e] = (r + e < rhi) ? col[e] : 0.0;
            }
        }
    };
    if (!masked && !ymode) {
        // Full slices without checks: a P row past pw reads row pw - 1 of Y and a
        // column past nt column nt - 1 of C, stored as zeros.
        const int64_t colq_max = nt - 1;
        auto faf = [&](int p, int64_t k, double (&v)[VA]) {
            load_run(A + (j0 + (p < pw ? p : pw - 1)) * lda + rlo + k, v);
            return p >= pw;
        };
        auto fbf = [&](int qi, int64_t k, double (&v)[VB]) {
            const int64_t q = q0 + qi;
            load_run(A + (c0 + (q < nt ? q : colq_max)) * lda + rlo + k, v);
            return q >= nt;
        };
        gemm_tile_runs_ft<WS, true, true>(acc, lds, rhi - rlo, faf, fbf, fa, fb);
    } else {
        gemm_tile_runs<WS, true, true>(acc, lds, rhi - rlo, fa, fb);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WS::WN, wn = wave % WS::WN;
    double *P = w.wpart + (ch * OB2 + prow0) * w.wp_ld;
#pragma unroll
    for (int i = 0; i < WS::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < WS::FN; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = acc_row<WS>(wm, i, lane, e);
                const int64_t q = q0 + acc_col<WS>(wn, jj, lane, e);
                if (p < pw && q < nt)
                    P[p * w.wp_ld + q] = acc[i][jj][e];
            }
}

// W[p][q] = sum_{s <= p} T[s][p] sum_ch P[ch][s][q] (T upper triangular,
// row-major with leading dimension tld); 64 columns per workgroup, thread
// (q, part) handles panel rows p = part, part + 4, ...  The chunk partials
// are summed in a fixed order (chunks ch = 0, 2, ... and 1, 3, ... then the
// two sums); T is staged in LDS as its packed upper triangle.
template <class TW>
__global__ __launch_bounds__(256) void qr_wred_kernel(QrWork w, const double *__restrict__ T, int tld, int pw,
                                                      int64_t nch, int64_t nt, TW *__restrict__ Wout, int prow0)
{
    __shared__ double Pm[OB][64 + 1];
    __shared__ double Tt[OB * (OB + 1) / 2];  // column p at p (p + 1) / 2 holds T[0..p][p]
    const int t = threadIdx.x;
    const int ql = t & 63, part = t >> 6;
    const int64_t q = (int64_t)blockIdx.x * 64 + ql;
    {
        double tv[OB * OB / 256];
#pragma unroll
        for (int u = 0; u < OB * OB / 256; ++u) {
            const int idx = t + 256 * u, r = idx / OB, p = idx % OB;
            tv[u] = (r <= p && p < pw) ? T[r * tld + p] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < OB * OB / 256; ++u) {
            const int idx = t + 256 * u, r = idx / OB, p = idx % OB;
            if (r <= p)
                Tt[p * (p + 1) / 2 + r] = tv[u];
        }
    }
    for (int p = part; p < pw; p += 4) {
        double s0 = 0.0, s1 = 0.0;
        if (q < nt) {
            const double *src = w.wpart + (prow0 + p) * w.wp_ld + q;
            const int64_t step = (int64_t)OB2 * w.wp_ld;
            int64_t ch = 0;
            for (; ch + 1 < nch; ch += 2) {
                s0 += src[ch * step];
                s1 += src[(ch + 1) * step];
            }
            if (ch < nch)
                s0 += src[ch * step];
        }
        Pm[p][ql] = s0 + s1;
    }
    __syncthreads();
    if (q >= nt)
        return;
    for (int p = part; p < pw; p += 4) {
        const double *tc = Tt + p * (p + 1) / 2;
        double s = 0.0;
        for (int r = 0; r <= p; ++r)
            s += tc[r] * Pm[r][ql];
        Wout[(prow0 + p) * w.ldw + q] = (TW)s;
    }
}

// Sum of the split-K partials over the row chunks into chunk 0's slot, one
// (p, q) element per thread (qr_wred_kernel's fixed order: even chunks, odd
// chunks, then the two sums).  qr_wred_kernel then reads a single chunk: its
// own reduction runs on only ceil(nt / 64) workgroups, two for the next
// block's columns.
__global__ __launch_bounds__(256) void qr_psum_kernel(QrWork w, int pw, int64_t nch, int64_t nt)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)pw * nt)
        return;
    const int64_t p = e / nt, q = e % nt;
    double *src = w.wpart + p * w.wp_ld + q;
    const int64_t step = (int64_t)OB2 * w.wp_ld;
    double s0 = 0.0, s1 = 0.0;
    int64_t ch = 0;
#pragma unroll 4
    for (; ch + 1 < nch; ch += 2) {
        s0 += src[ch * step];
        s1 += src[(ch + 1) * step];
    }
    if (ch < nch)
        s0 += src[ch * step];
    src[0] = s0 + s1;
}

// G = Y_A^T Y_B from the chunk partials (one entry per thread: ld x ld
// entries, rows p < ld of the partials, columns q < pwb, G row-major with leading
// dimension ld; chunks summed in the same fixed order as qr_wred_kernel).
__global__ __launch_bounds__(256) void qr_gsum_kernel(QrWork w, int pwb, int64_t nch, double *__restrict__ G, int ld)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= ld * ld)
        return;
    const int p = e / ld, q = e % ld;
    double s0 = 0.0, s1 = 0.0;
    if (q < pwb) {
        const double *src = w.wpart + p * w.wp_ld + q;
        const int64_t step = (int64_t)OB2 * w.wp_ld;
        int64_t ch = 0;
        for (; ch + 1 < nch; ch += 2) {
            s0 += src[ch * step];
            s1 += src[(ch + 1) * step];
        }
        if (ch < nch)
            s0 += src[ch * step];
    }
    G[e] = s0 + s1;
}

// Combined compact-WY factor of two consecutive panels A | B:
// T = [[T_A, -T_A G T_B], [0, T_B]] with G = Y_A^T Y_B (summed by qr_gsum_kernel).
__global__ __launch_bounds__(256) void qr_tcombine_kernel(QrWork w, const double *__restrict__ Gs,
                                                         double *__restrict__ Tout)
{
    __shared__ double TA[NB][NB + 1];
    __shared__ double TB[NB][NB + 1];
    __shared__ double G[NB][NB + 1];
    __shared__ double X[NB][NB + 1];
    const int t = threadIdx.x;
    const double *Ta = w.Tin, *Tb = w.Tin + NB * NB;
    {
        double a[16], b[16], g[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            a[u] = Ta[t + 256 * u];
            b[u] = Tb[t + 256 * u];
            g[u] = Gs[t + 256 * u];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int idx = t + 256 * u, r = idx / NB, c = idx % NB;
            TA[r][c] = a[u];
            TB[r][c] = b[u];
            G[r][c] = g[u];
        }
    }
    __syncthreads();
    for (int idx = t; idx < NB * NB; idx += 256) {  // X = G T_B
        const int r = idx / NB, c = idx % NB;
        double v = 0.0;
        for (int k = 0; k <= c; ++k)
            v += G[r][k] * TB[k][c];
        X[r][c] = v;
    }
    __syncthreads();
    for (int idx = t; idx < OB * OB; idx += 256) {
        const int r = idx / OB, c = idx % OB;
        double v = 0.0;
        if (r < NB && c < NB) {
            v = TA[r][c];
        } else if (r >= NB && c >= NB) {
            v = TB[r - NB][c - NB];
        } else if (r < NB && c >= NB) {  // -T_A X
            const int cc = c - NB;
            for (int k = r; k < NB; ++k)
                v -= TA[r][k] * X[k][cc];
        }
        Tout[idx] = v;
    }
}

// ---------------------------------------------------------------------------
// A trailing-update block of two panel pairs a | b (up to 256 columns).  Its
// compact-WY factor is T = [[T_a, -T_a G T_b], [0, T_b]] with G = Y_a^T Y_b, so
// W = T^T P for P = Y^T C splits into W_a = T_a^T P_a and
// W_b = T_b^T (P_b - H^T P_a) with H = T_a G: the two 128-row halves reuse the
// 128-column reduction, and the update C -= Y W runs once with depth 256.
// ---------------------------------------------------------------------------

// H = T_a G (T_a upper triangular pwa x pwa, row-major ld tld; G and H
// row-major, leading dimension OB; columns q < pwb).  Grid OB: workgroup i
// forms row i, one column per thread.
__global__ __launch_bounds__(OB) void qr_hmat_kernel(const double *__restrict__ Ta, int tld, int pwa,
                                                     const double *__restrict__ G, int pwb, double *__restrict__ H)
{
    const int i = blockIdx.x, j = threadIdx.x;
    double v = 0.0;
    if (i < pwa && j < pwb)
        for (int k = i; k < pwa; ++k)
            v += Ta[i * tld + k] * G[k * OB + j];
    H[i * OB + j] = v;
}

// P_b -= H^T P_a on the summed partials (chunk 0): P rows OB + p, p < pwb, columns
// q < nt.  Workgroup (x, y) takes 64 columns and the 32 rows p of quarter y, with
// P_a (rows s < pwa) and H's 32 columns staged in LDS; thread (q, part) forms
// rows p = 32 y + 8 part .. + 7.
constexpr int PC_ROWS = 32;
__global__ __launch_bounds__(256) void qr_pcorr_kernel(QrWork w, const double *__restrict__ H, int pwa, int pwb,
                                                       int64_t nt)
{
    __shared__ double Pa[OB][64];
    __shared__ double Hs[OB][PC_ROWS];
    const int t = threadIdx.x, ql = t & 63, part = t >> 6;
    const int p0 = PC_ROWS * (int)blockIdx.y;
    if (p0 >= pwb)
        return;
    const int64_t q = (int64_t)blockIdx.x * 64 + ql;
    for (int sr = part; sr < OB; sr += 4)
        Pa[sr][ql] = (sr < pwa && q < nt) ? w.wpart[sr * w.wp_ld + q] : 0.0;
    for (int e = t; e < OB * PC_ROWS; e += 256) {
        const int sr = e / PC_ROWS, pp = e % PC_ROWS;
        Hs[sr][pp] = sr < pwa ? H[sr * OB + p0 + pp] : 0.0;
    }
    __syncthreads();
    if (q >= nt)
        return;
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
        acc[u] = 0.0;
    for (int sr = 0; sr < pwa; ++sr) {
        const double a = Pa[sr][ql];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            acc[u] += Hs[sr][8 * part + u] * a;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int p = p0 + 8 * part + u;
        if (p < pwb)
            w.wpart[(OB + p) * w.wp_ld + q] -= acc[u];
    }
}

// Copy a pw x pw row-major T (leading dimension sld) into dst (leading dimension OB).
__global__ __launch_bounds__(256) void qr_tcopy_kernel(const double *__restrict__ src, int sld, int pw,
                                                       double *__restrict__ dst)
{
    for (int e = threadIdx.x; e < OB * OB; e += 256) {
        const int i = e / OB, j = e % OB;
        dst[e] = (i < pw && j < pw) ? src[i * sld + j] : 0.0;
    }
}

// C[r][q] -= sum_p Y[r][p] W[p][q] for rows j0.. and columns c0 .. c0+nt; the
// tile is computed transposed so that consecutive lanes write consecutive rows.
// The accumulators start from the C tile (its loads in flight with the first
// operand slices) and take -W, so the epilogue is a plain store.
template <int PART>
__global__ __launch_bounds__(256, 3) void qr_update_kernel(QrWork w, int64_t j0, int pw, int64_t c0, int64_t nt,
                                                          int n_head)
{
    __shared__ double lds[2 * US::STAGE];
    int64_t rb, cb;
    if (!update_tile_part<PART>((w.m - j0 + US::BN - 1) / US::BN, (nt + US::BM - 1) / US::BM, n_head, rb,
                                cb))
        return;
    const int64_t q0 = cb * US::BM;
    const int64_t r0 = j0 + rb * US::BN;
    const double *A = w.A;
    const int64_t lda = w.lda, m = w.m, ldW = w.ldw;
    const double *W = w.W;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / US::WN, wn = wave % US::WN;
    double *C = w.A + c0 * lda;
    d4 acc[US::FM][US::FN];
#pragma unroll
    for (int i = 0; i < US::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < US::FN; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t q = q0 + acc_row<US>(wm, i, lane, e);
                const int64_t r = r0 + acc_col<US>(wn, jj, lane, e);
                acc[i][jj][e] = ((PART == 1 || r < m) && q < nt) ? C[q * lda + r] : 0.0;
            }
    const bool masked = r0 < j0 + pw;  // the row block meets Y's unit upper triangle
    constexpr int VA = US::BM * US::BK / US::NT, VB = US::BN * US::BK / US::NT;
    auto fa = [&](int qi, int64_t p, double (&v)[VA]) {
        const int64_t q = q0 + qi;
        if (p >= pw) {
#pragma unroll
            for (int e = 0; e < VA; ++e)
                v[e] = 0.0;
        } else if (q + VA <= nt) {
            load_run(W + p * ldW + q, v);
#pragma unroll
            for (int e = 0; e < VA; ++e)
                v[e] = -v[e];
        } else {
#pragma unroll
            for (int e = 0; e < VA; ++e)
                v[e] = (q + e < nt) ? -W[p * ldW + q + e] : 0.0;
        }
    };
    auto fb = [&](int ri, int64_t p, double (&v)[VB]) {
        const int64_t r = r0 + ri;
        if (p >= pw) {
#pragma unroll
            for (int e = 0; e < VB; ++e)
                v[e] = 0.0;
        } else if (PART == 1 || (!masked && r + VB <= m)) {
            load_run(A + (j0 + p) * lda + r, v);
        } else {
#pragma unroll
            for (int e = 0; e < VB; ++e)
                v[e] = ypanel(A, lda, m, j0, pw, r + e, (int)p);
        }
    };
    gemm_tile_runs<US, false, false>(acc, lds, pw, fa, fb);
    // recompute the store addresses rather than keep the loads' live through the product
    int64_t q0s = q0, r0s = r0;
    asm volatile("" : "+s"(q0s), "+s"(r0s));
#pragma unroll
    for (int i = 0; i < US::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < US::FN; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t q = q0s + acc_row<US>(wm, i, lane, e);
                const int64_t r = r0s + acc_col<US>(wn, jj, lane, e);
                if ((PART == 1 || r < m) && q < nt)
                    C[q * lda + r] = acc[i][jj][e];
            }
}

using WS32 = TileShape<OB, 128, 16, 2, 2>;   // FP32 P = Y^T C (16-deep: four waves per SIMD)
using US32 = TileShape<128, 128, 16, 2, 2>;  // FP32 C^T -= W^T Y^T (16-deep: three waves per SIMD)

// FP32-storage versions of qr_wpart_kernel / qr_update_kernel on FP32 MFMA.
__global__ __launch_bounds__(256, 3) void qr_wpart32_kernel(QrWork w, int64_t j0, int pw, int64_t c0, int64_t nt,
                                                            int ymode, int64_t r0, int64_t chunk)
{
    __shared__ float lds[2 * WS32::STAGE];
    const int prow0 = OB * (int)blockIdx.z;
    j0 += prow0;
    pw = (pw - prow0) < OB ? (pw - prow0) : OB;
    if (pw <= 0)
        return;
    const int64_t ch = blockIdx.y;
    const int64_t q0 = (int64_t)blockIdx.x * WS32::BN;
    const int64_t rlo = r0 + ch * chunk;
    int64_t rhi = rlo + chunk;
    if (rhi > w.m)
        rhi = w.m;
    if (rlo >= rhi)
        return;
    f4 acc[WS32::FM][WS32::FN];
    zero_acc32<WS32>(acc);
    const float *A = w.A32;
    const int64_t lda = w.lda, m = w.m;
    const bool masked = rlo < j0 + pw;
    constexpr int VA = WS32::BM * WS32::BK / WS32::NT, VB = WS32::BN * WS32::BK / WS32::NT;
    auto fa = [&](int p, int64_t k, float (&v)[VA]) {
        const int64_t r = rlo + k;
        if (p >= pw) {
#pragma unroll
            for (int e = 0; e < VA; ++e)
                v[e] = 0.0f;
        } else if (!masked && r + VA <= rhi) {
            load_run(A + (j0 + p) * lda + r, v);
        } else {
#pragma unroll
            for (int e = 0; e < VA; ++e)
                v[e] = (r + e < rhi) ? ypanel(A, lda, m, j0, pw, r + e, p) : 0.0f;
        }
    };
    auto fb = [&](int qi, int64_t k, float (&v)[VB]) {
        const int64_t r = rlo + k, q = q0 + qi;
        if (q >= nt) {
#pragma unroll
            for (int e = 0; e < VB; ++e)
                v[e] = 0.0f;
        } else if (ymode) {
#pragma unroll
            for (int e = 0; e < VB; ++e)
                v[e] = (r + e < rhi) ? ypanel(A, lda, m, c0, (int)nt, r + e, (int)q) : 0.0f;
        } else {
            const float *col = A + (c0 + q) * lda + r;
            if (r + VB <= rhi) {
                load_run(col, v);
            } else {
#pragma unroll
                for (int e = 0; e < VB; ++e)
                    v[e] = (r + e < rhi) ? col[e] : 0.0f;
            }
        }
    };
    gemm_tile_runs32<WS32, true, true>(acc, lds, rhi - rlo, fa, fb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WS32::WN, wn = wave % WS32::WN;
    double *P = w.wpart + (ch * OB2 + prow0) * w.wp_ld;
#pragma unroll
    for (int i = 0; i < WS32::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < WS32::FN; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = acc32_row<WS32>(wm, i, lane, e);
                const int64_t q = q0 + acc32_col<WS32>(wn, jj, lane, e);
                if (p < pw && q < nt)
                    P[p * w.wp_ld + q] = (double)acc[i][jj][e];
            }
}

template <int PART>
__global__ __launch_bounds__(256, 3) void qr_update32_kernel(QrWork w, int64_t j0, int pw, int64_t c0, int64_t nt,
                                                          int n_head)
{
    __shared__ float lds[2 * US32::STAGE];
    int64_t rb, cb;
    if (!update_tile_part<PART>((w.m - j0 + US32::BN - 1) / US32::BN, (nt + US32::BM - 1) / US32::BM, n_head, rb,
                                cb))
        return;
    const int64_t q0 = cb * US32::BM;
    const int64_t r0 = j0 + rb * US32::BN;
    const float *A = w.A32;
    const int64_t lda = w.lda, m = w.m, ldW = w.ldw;
    const float *W = w.W32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / US32::WN, wn = wave % US32::WN;
    float *C = w.A32 + c0 * lda;
    f4 acc[US32::FM][US32::FN];  // starts from the C tile; the product takes -W
#pragma unroll
    for (int i = 0; i < US32::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < US32::FN; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t q = q0 + acc32_row<US32>(wm, i, lane, e);
                const int64_t r = r0 + acc32_col<US32>(wn, jj, lane, e);
                acc[i][jj][e] = ((PART == 1 || r < m) && q < nt) ? C[q * lda + r] : 0.0f;
            }
    const bool masked = r0 < j0 + pw;
    constexpr int VA = US32::BM * US32::BK / US32::NT, VB = US32::BN * US32::BK / US32::NT;
    auto fa = [&](int qi, int64_t p, float (&v)[VA]) {
        const int64_t q = q0 + qi;
        if (p >= pw) {
#pragma unroll
            for (int e = 0; e < VA; ++e)
                v[e] = 0.0f;
        } else if (q + VA <= nt) {
            load_run(W + p * ldW + q, v);
#pragma unroll
            for (int e = 0; e < VA; ++e)
                v[e] = -v[e];
        } else {
#pragma unroll
            for (int e = 0; e < VA; ++e)
                v[e] = (q + e < nt) ? -W[p * ldW + q + e] : 0.0f;
        }
    };
    auto fb = [&](int ri, int64_t p, float (&v)[VB]) {
        const int64_t r = r0 + ri;
        if (p >= pw) {
#pragma unroll
            for (int e = 0; e < VB; ++e)
                v[e] = 0.0f;
        } else if (PART == 1 || (!masked && r + VB <= m)) {
            load_run(A + (j0 + p) * lda + r, v);
        } else {
#pragma unroll
            for (int e = 0; e < VB; ++e)
                v[e] = ypanel(A, lda, m, j0, pw, r + e, (int)p);
        }
    };
    gemm_tile_runs32<US32, false, false>(acc, lds, pw, fa, fb);
    int64_t q0s = q0, r0s = r0;
    asm volatile("" : "+s"(q0s), "+s"(r0s));
#pragma unroll
    for (int i = 0; i < US32::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < US32::FN; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t q = q0s + acc32_row<US32>(wm, i, lane, e);
                const int64_t r = r0s + acc32_col<US32>(wn, jj, lane, e);
                if ((PART == 1 || r < m) && q < nt)
                    C[q * lda + r] = acc[i][jj][e];
            }
}

// Split of rows [r0, m) into chunks for the split-K products.
static void chunking(int64_t rows, int64_t ncb, int64_t &chunk, int64_t &nch, int64_t cap, int64_t target = 2048)
{
    nch = (target + ncb - 1) / ncb;
    if (nch > cap)
        nch = cap;
    chunk = (rows + nch - 1) / nch;
    chunk = (chunk + 15) & ~int64_t(15);
    if (chunk < 256)
        chunk = 256;
    nch = (rows + chunk - 1) / chunk;
}

// w with its rows cut to those that can be nonzero in columns [0, j_end): below a
// trailing upper-triangular block's row tri0 + j_end, every column before j_end
// is still zero, so the reflectors of those columns are zero there and leave
// those rows unchanged.
static QrWork rows_to(const QrWork &w, int64_t j_end)
{
    QrWork r = w;
    if (w.tri0 > 0 && w.tri0 + j_end < w.m)
        r.m = w.tri0 + j_end;
    return r;
}

// TSQR + reconstruction of the panel at (j0, j0) of width pw; its T goes to Tout.
template <class T>
static void factor_panel(const QrWork &wf, int64_t j0, int pw, double *Tout, hipStream_t s)
{
    const QrWork w = rows_to(wf, j0 + pw);
    if (w.panel == 0) {
        if constexpr (sizeof(T) == 8)
            cqr_panel_f64(w, j0, pw, Tout, s);
        else
            cqr_panel_f32(w, j0, pw, Tout, s);
        return;
    }
    const int64_t mk = w.m - j0;
    const PanelTree pt = panel_tree(mk);
    for (int l = 0; l < pt.levels; ++l)
        hipLaunchKernelGGL(tsqr_factor_kernel<T>, dim3((unsigned)pt.nodes[l]), dim3(TS_NT), 0, s, w, j0, pw, l,
                           pt.nodes[l], l > 0 ? pt.nodes[l - 1] : 0, mk);
    for (int l = pt.levels - 1; l >= 0; --l)
        hipLaunchKernelGGL(tsqr_formq_kernel<T>, dim3((unsigned)pt.nodes[l]), dim3(TS_NT), 0, s, w, j0, pw, l,
                           pt.nodes[l], l == pt.levels - 1 ? 1 : 0, mk);
    hipLaunchKernelGGL(tsqr_lu_kernel<T>, dim3(1), dim3(256), 0, s, w, j0, pw, pt.levels - 1, Tout);
    if (mk > pw)
        hipLaunchKernelGGL(tsqr_trsm_kernel<T>, dim3((unsigned)((mk - pw + 255) / 256)), dim3(256), 0, s, w, j0,
                           pw);
}

// P = Y^T C (split over row chunks) for the block at (j0, j0) of width pw.
template <class T>
static void launch_wpart(const QrWork &w, int64_t j0, int pw, int64_t c0, int64_t nt, int ymode, int64_t r0,
                         int64_t chunk, int64_t ncb, int64_t nch, int halves, hipStream_t s)
{
    if constexpr (sizeof(T) == 8)
        hipLaunchKernelGGL(qr_wpart_kernel, dim3((unsigned)ncb, (unsigned)nch, (unsigned)halves), dim3(256), 0, s, w,
                           j0, pw, c0, nt, ymode, r0, chunk);
    else
        hipLaunchKernelGGL(qr_wpart32_kernel, dim3((unsigned)ncb, (unsigned)nch, (unsigned)halves), dim3(256), 0, s,
                           w, j0, pw, c0, nt, ymode, r0, chunk);
}

// The compact-WY data of a trailing-update block at column J: panel pair a
// (pwa <= OB columns, T_a) and, when present, pair b (pwb columns, T_b) with
// H = T_a Y_a^T Y_b.  Storage: four OB x OB row-major matrices (Ta, Tb, G, H).
struct BlockT {
    double *store;
    int pwa = 0, pwb = 0;
    const double *ta = nullptr;  // T_a as apply_block reads it (row-major, ld tld); null: Ta()
    int tld = OB;
    double *Ta() const { return store; }
    double *Tb() const { return store + OB * OB; }
    double *G() const { return store + 2 * OB * OB; }
    double *H() const { return store + 3 * OB * OB; }
    int pw() const { return pwa + pwb; }
};

// C := (I - Y T Y^T)^T C for the columns c0 .. c0+nt, Y the block at (J, J).
template <class T>
static void apply_block(const QrWork &wf, int64_t J, const BlockT &bt, int64_t c0, int64_t nt, hipStream_t s)
{
    if (nt <= 0)
        return;
    const int pw = bt.pw();
    const QrWork w = rows_to(wf, J + pw);
    const int64_t rows = w.m - J;
    const int64_t ncb = (nt + WS::BN - 1) / WS::BN;
    int64_t chunk, nch;
    const int halves = bt.pwb > 0 ? 2 : 1;  // 128-row halves of P, one grid layer each
    chunking(rows, ncb * halves, chunk, nch, w.max_chunks, w.split_wgs > 0 ? w.split_wgs : 2048);
    launch_wpart<T>(w, J, pw, c0, nt, 0, J, chunk, ncb, nch, halves, s);
    if (nch > 1) {
        hipLaunchKernelGGL(qr_psum_kernel, dim3((unsigned)(((int64_t)pw * nt + 255) / 256)), dim3(256), 0, s, w, pw,
                           nch, nt);
        nch = 1;
    }
    const unsigned gq = (unsigned)((nt + 63) / 64);
    const double *ta = bt.ta ? bt.ta : bt.Ta();
    const int tld = bt.ta ? bt.tld : OB;
    if constexpr (sizeof(T) == 8) {
        hipLaunchKernelGGL(qr_wred_kernel<double>, dim3(gq), dim3(256), 0, s, w, ta, tld, bt.pwa, nch, nt, w.W, 0);
        if (bt.pwb > 0) {
            hipLaunchKernelGGL(qr_pcorr_kernel, dim3(gq, OB / PC_ROWS), dim3(256), 0, s, w, (const double *)bt.H(),
                               bt.pwa, bt.pwb, nt);
            hipLaunchKernelGGL(qr_wred_kernel<double>, dim3(gq), dim3(256), 0, s, w, (const double *)bt.Tb(), OB,
                               bt.pwb, nch, nt, w.W, OB);
        }
    } else {
        hipLaunchKernelGGL(qr_wred_kernel<float>, dim3(gq), dim3(256), 0, s, w, ta, tld, bt.pwa, nch, nt, w.W32,
                           0);
        if (bt.pwb > 0) {
            hipLaunchKernelGGL(qr_pcorr_kernel, dim3(gq, OB / PC_ROWS), dim3(256), 0, s, w, (const double *)bt.H(),
                               bt.pwa, bt.pwb, nt);
            hipLaunchKernelGGL(qr_wred_kernel<float>, dim3(gq), dim3(256), 0, s, w, (const double *)bt.Tb(), OB,
                               bt.pwb, nch, nt, w.W32, OB);
        }
    }
    const int n_head = (pw + US::BN - 1) / US::BN;  // row blocks of 128 that meet Y's unit triangle
    static_assert(US::BN == US32::BN, "one row-block split for both update kernels");
    auto grid = [](int64_t tiles) { return dim3((unsigned)((tiles + 7) & ~int64_t(7))); };
    if constexpr (sizeof(T) == 8) {
        const int64_t nrb = (rows + US::BN - 1) / US::BN, ncb_u = (nt + US::BM - 1) / US::BM;
        if (nrb > n_head + 1) {  // interior row blocks without checks, then the edge ones
            hipLaunchKernelGGL(qr_update_kernel<1>, grid((nrb - n_head - 1) * ncb_u), dim3(256), 0, s, w, J, pw, c0,
                               nt, n_head);
            hipLaunchKernelGGL(qr_update_kernel<2>, grid((n_head + 1) * ncb_u), dim3(256), 0, s, w, J, pw, c0, nt,
                               n_head);
        } else {
            hipLaunchKernelGGL(qr_update_kernel<0>, grid(nrb * ncb_u), dim3(256), 0, s, w, J, pw, c0, nt, n_head);
        }
    } else {
        const int64_t nrb = (rows + US32::BN - 1) / US32::BN, ncb_u = (nt + US32::BM - 1) / US32::BM;
        if (nrb > n_head + 1) {
            hipLaunchKernelGGL(qr_update32_kernel<1>, grid((nrb - n_head - 1) * ncb_u), dim3(256), 0, s, w, J, pw,
                               c0, nt, n_head);
            hipLaunchKernelGGL(qr_update32_kernel<2>, grid((n_head + 1) * ncb_u), dim3(256), 0, s, w, J, pw, c0, nt,
                               n_head);
        } else {
            hipLaunchKernelGGL(qr_update32_kernel<0>, grid(nrb * ncb_u), dim3(256), 0, s, w, J, pw, c0, nt, n_head);
        }
    }
}

// Factor the panel pair at column J (main-stream scratch in w): panel A, its
// update of panel B, panel B, and the pair's compact-WY T (row-major, copied
// to Tdst with leading dimension OB).  Returns the pair's width.
template <class T>
static int factor_pair(const QrWork &w, int64_t J, double *Tdst, hipStream_t s)
{
    double *Ta = w.Tin, *Tb = w.Tin + NB * NB;
    const int pwa = (int)((w.n - J) < NB ? (w.n - J) : NB);
    factor_panel<T>(w, J, pwa, Ta, s);
    const int64_t jb = J + pwa;
    const int pwb = (int)((w.n - jb) < NB ? (w.n - jb) : NB);
    if (pwb <= 0) {
        hipLaunchKernelGGL(qr_tcopy_kernel, dim3(1), dim3(256), 0, s, (const double *)Ta, NB, pwa, Tdst);
        return pwa;
    }
    BlockT pa{nullptr, pwa, 0, Ta, NB};  // panel A alone
    apply_block<T>(w, J, pa, jb, pwb, s);
    factor_panel<T>(w, jb, pwb, Tb, s);
    const QrWork wg = rows_to(w, jb + pwb);  // G = Y_a^T Y_b
    const int64_t rows = wg.m - jb;
    int64_t chunk, nch;
    chunking(rows, 1, chunk, nch, wg.max_chunks);
    launch_wpart<T>(wg, J, pwa, jb, (int64_t)pwb, 1, jb, chunk, 1, nch, 1, s);
    hipLaunchKernelGGL(qr_gsum_kernel, dim3(NB * NB / 256), dim3(256), 0, s, wg, pwb, nch, wg.cq_G, NB);
    hipLaunchKernelGGL(qr_tcombine_kernel, dim3(1), dim3(256), 0, s, w, (const double *)w.cq_G, Tdst);
    return pwa + pwb;
}

// Factor the trailing-update block at column J: panel pair a, its update of
// pair b's columns, pair b, then G = Y_a^T Y_b and H = T_a G.  bt.store holds the
// results; returns the block's width (up to OB2).
template <class T>
static int factor_block(const QrWork &w, int64_t J, BlockT &bt, hipStream_t s)
{
    bt.pwa = factor_pair<T>(w, J, bt.Ta(), s);
    bt.pwb = 0;
    const int64_t jb = J + bt.pwa;
    const int pwb_max = (int)((w.n - jb) < OB ? (w.n - jb) : OB);
    if (bt.pwa < OB || pwb_max <= 0)
        return bt.pwa;
    BlockT a{bt.store, bt.pwa, 0};
    apply_block<T>(w, J, a, jb, pwb_max, s);
    bt.pwb = factor_pair<T>(w, jb, bt.Tb(), s);
    const QrWork wg = rows_to(w, jb + bt.pwb);  // G = Y_a^T Y_b
    const int64_t rows = wg.m - jb;
    int64_t chunk, nch;
    chunking(rows, 1, chunk, nch, wg.max_chunks);
    launch_wpart<T>(wg, J, bt.pwa, jb, (int64_t)bt.pwb, 1, jb, chunk, 1, nch, 1, s);
    hipLaunchKernelGGL(qr_gsum_kernel, dim3(OB * OB / 256), dim3(256), 0, s, wg, bt.pwb, nch, bt.G(), OB);
    hipLaunchKernelGGL(qr_hmat_kernel, dim3(OB), dim3(OB), 0, s, (const double *)bt.Ta(), OB, bt.pwa,
                       (const double *)bt.G(), bt.pwb, bt.H());
    return bt.pw();
}

template <class T>
static void geqrf(const QrWork &w, hipStream_t s, const QrAsync *la)
{
    // small-scratch views: wn for the products inside a block (at most OB rows
    // and columns of P), wm for the main stream's update of the next block (OB2)
    QrWork wn = w;
    wn.wpart = w.wpart_s;
    wn.wp_ld = OB;
    wn.W = w.W_s;
    wn.W32 = w.W32_s;
    wn.ldw = OB;
    wn.max_chunks = MAX_CHUNKS_S;  // more row chunks keep the panel chain's GEMMs wide
    QrWork wm = wn;
    wm.wp_ld = OB2;
    wm.ldw = OB2;
    wm.max_chunks = MAX_CHUNKS_S / 2;  // same buffer
    if (!la) {
        BlockT bt{w.T};
        for (int64_t J = 0; J < w.n; J += bt.pw()) {
            factor_block<T>(wn, J, bt, s);
            apply_block<T>(w, J, bt, J + bt.pw(), w.ncols - (J + bt.pw()), s);
        }
        return;
    }
    BlockT bt[2] = {BlockT{w.T}, BlockT{w.T2}};
    (void)hipEventRecord(la->fork, s);
    (void)hipStreamWaitEvent(la->side, la->fork, 0);
    factor_block<T>(wn, 0, bt[0], s);
    (void)hipEventRecord(la->t_ready, s);
    int64_t k = 0;
    for (int64_t J = 0; J < w.n; ++k) {
        const BlockT &cur = bt[k & 1];
        const int64_t cn = J + cur.pw();                          // first column of block k+1
        const int64_t nn = (w.n - cn) < OB2 ? (w.n - cn) : OB2;   // its width (0 after the last block)
        // side: block k's update of everything right of block k+1 (b included)
        (void)hipStreamWaitEvent(la->side, la->t_ready, 0);
        apply_block<T>(w, J, cur, cn + nn, w.ncols - (cn + nn), la->side);
        (void)hipEventRecord(la->bulk[k & 1], la->side);
        if (nn <= 0)
            break;
        // main: block k+1's columns need every earlier block's update first; its
        // T buffer is the one block k-1's side update read
        if (k > 0)
            (void)hipStreamWaitEvent(s, la->bulk[(k - 1) & 1], 0);
        apply_block<T>(wm, J, cur, cn, nn, s);
        factor_block<T>(wn, cn, bt[(k + 1) & 1], s);
        (void)hipEventRecord(la->t_ready, s);
        J = cn;
    }
    (void)hipEventRecord(la->join, la->side);
    (void)hipStreamWaitEvent(s, la->join, 0);
}

hipError_t launch_geqrf(const QrWork &w, hipStream_t s, const QrAsync *la)
{
    if (w.A32)
        geqrf<float>(w, s, la);
    else
        geqrf<double>(w, s, la);
    return hipGetLastError();
}

}  // namespace gap
