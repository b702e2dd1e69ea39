// Blocked Householder QR of the augmented stacked matrix [A | b] in FP64
// (Sec. Implementation: the factorisation leaves R in the upper triangle and
// the Householder vectors below it with their weights tau; Q^T b comes from
// carrying b along as an extra column, which is what applying the stored
// reflectors to b computes).
//
// Each 64-column panel is factored as a tall-skinny QR (TSQR) over a
// 4-ary tree of 256-row tiles, its explicit Q formed top-down, and the
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
constexpr int64_t MAX_CHUNKS = 64;

int64_t qr_max_chunks() { return MAX_CHUNKS; }

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
        const double *col = w.A + (j0 + q) * w.lda + j0 + lo;
        const int64_t nr = hi - lo;
#pragma unroll
        for (int i = 0; i < SLOTS; ++i) {
            const int r = NPART * i + part;
            x[i] = (q < pw && r < nr) ? col[r] : 0.0;
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
            double *col = w.A + (j0 + q) * w.lda + j0 + lo;
            const int64_t nr = hi - lo;
#pragma unroll
            for (int i = 0; i < SLOTS; ++i) {
                const int r = NPART * i + part;
                if (r < nr)
                    col[r] = x[i];
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
__global__ __launch_bounds__(256) void tsqr_lu_kernel(QrWork w, int64_t j0, int pw, int root_level)
{
    __shared__ double B[NB][NB + 1];
    __shared__ double Z[NB][NB + 1];
    __shared__ double sg[NB];
    const int t = threadIdx.x;
    for (int idx = t; idx < pw * pw; idx += 256) {
        const int r = idx % pw, c = idx / pw;
        B[r][c] = w.A[(j0 + c) * w.lda + j0 + r];
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
        w.T[idx] = tv;
        w.U[idx] = (r < pw && c < pw && r <= c) ? B[r][c] : 0.0;
        if (r < pw && c < pw) {
            double out;
            if (r <= c)
                out = sg[r] * root[c * TR + r];
            else
                out = B[r][c];
            w.A[(j0 + c) * w.lda + j0 + r] = out;
        }
        if (r == c && r < pw)
            w.tau[j0 + r] = tv;
    }
}

// Rows below the top block: Y = Q U^-1 (one row per thread).
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
        y[c] = (c < pw) ? w.A[(j0 + c) * w.lda + r] : 0.0;
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
            w.A[(j0 + c) * w.lda + r] = y[c];
}

// Householder vectors of the panel at (j0, j0): unit lower trapezoidal.
DEV double ypanel(const double *A, int64_t lda, int64_t m, int64_t j0, int pw, int64_t r, int p)
{
    if (p >= pw || r >= m)
        return 0.0;
    const int64_t d = r - (j0 + p);
    if (d < 0)
        return 0.0;
    if (d == 0)
        return 1.0;
    return A[(j0 + p) * lda + r];
}

using WS = TileShape<NB, 128, 16, 1, 4>;   // P = Y^T C, split over row chunks
using US = TileShape<128, 128, 16, 2, 2>;  // C^T -= W^T Y^T (rows of C along the MFMA N axis)

// P[ch][p][q] = sum over the chunk's rows r of Y[r][p] C[r][q], C = columns j0+pw..
__global__ __launch_bounds__(256) void qr_wpart_kernel(QrWork w, int64_t j0, int pw, int64_t chunk, int64_t nt)
{
    __shared__ double lds[2 * WS::STAGE];
    const int64_t ch = blockIdx.y;
    const int64_t q0 = (int64_t)blockIdx.x * WS::BN;
    const int64_t rlo = j0 + ch * chunk;
    int64_t rhi = rlo + chunk;
    if (rhi > w.m)
        rhi = w.m;
    if (rlo >= rhi)
        return;
    d4 acc[WS::FM][WS::FN];
    zero_acc<WS>(acc);
    const double *A = w.A;
    const int64_t lda = w.lda, m = w.m;
    const double *C = A + (j0 + pw) * lda;
    auto fa = [&](int p, int64_t k) -> double {
        const int64_t r = rlo + k;
        return (r < rhi) ? ypanel(A, lda, m, j0, pw, r, p) : 0.0;
    };
    auto fb = [&](int qi, int64_t k) -> double {
        const int64_t r = rlo + k, q = q0 + qi;
        return (r < rhi && q < nt) ? C[q * lda + r] : 0.0;
    };
    gemm_tile<WS, true, true>(acc, lds, rhi - rlo, fa, fb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WS::WN, wn = wave % WS::WN;
    double *P = w.wpart + ch * NB * w.ncols;
#pragma unroll
    for (int i = 0; i < WS::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < WS::FN; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = acc_row<WS>(wm, i, lane, e);
                const int64_t q = q0 + acc_col<WS>(wn, jj, lane, e);
                if (q < nt)
                    P[p * w.ncols + q] = acc[i][jj][e];
            }
}

// W[p][q] = sum_{s <= p} T[s][p] sum_ch P[ch][s][q]; 64 columns per workgroup,
// thread (q, part) sums panel rows p = part, part + 4, ... over the chunks in order.
__global__ __launch_bounds__(256) void qr_wred_kernel(QrWork w, int pw, int64_t nch, int64_t nt)
{
    __shared__ double T[NB][NB + 1];
    __shared__ double Pm[NB][NB + 1];
    for (int idx = threadIdx.x; idx < NB * NB; idx += 256)
        T[idx / NB][idx % NB] = w.T[idx];
    const int ql = threadIdx.x & 63, part = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * NB + ql;
    for (int p = part; p < NB; p += 4) {
        double s = 0.0;
        if (p < pw && q < nt)
            for (int64_t ch = 0; ch < nch; ++ch)
                s += w.wpart[(ch * NB + p) * w.ncols + q];
        Pm[p][ql] = s;
    }
    __syncthreads();
    if (q >= nt)
        return;
    for (int p = part; p < NB; p += 4) {
        double s = 0.0;
        for (int r = 0; r <= p; ++r)
            s += T[r][p] * Pm[r][ql];
        w.W[p * w.ncols + q] = (p < pw) ? s : 0.0;
    }
}

// C[r][q] -= sum_p Y[r][p] W[p][q] for rows j0.. and columns j0+pw..; the tile
// is computed transposed so that consecutive lanes write consecutive rows.
__global__ __launch_bounds__(256) void qr_update_kernel(QrWork w, int64_t j0, int pw, int64_t nt)
{
    __shared__ double lds[2 * US::STAGE];
    const int64_t q0 = (int64_t)blockIdx.y * US::BM;
    const int64_t r0 = j0 + (int64_t)blockIdx.x * US::BN;
    const double *A = w.A;
    const int64_t lda = w.lda, m = w.m, ldW = w.ncols;
    const double *W = w.W;
    d4 acc[US::FM][US::FN];
    zero_acc<US>(acc);
    auto fa = [&](int qi, int64_t p) -> double {
        const int64_t q = q0 + qi;
        return (q < nt && p < pw) ? W[p * ldW + q] : 0.0;
    };
    auto fb = [&](int ri, int64_t p) -> double { return ypanel(A, lda, m, j0, pw, r0 + ri, (int)p); };
    gemm_tile<US, false, false>(acc, lds, pw, fa, fb);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / US::WN, wn = wave % US::WN;
    double *C = w.A + (j0 + pw) * lda;
#pragma unroll
    for (int i = 0; i < US::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < US::FN; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t q = q0 + acc_row<US>(wm, i, lane, e);
                const int64_t r = r0 + acc_col<US>(wn, jj, lane, e);
                if (r < m && q < nt)
                    C[q * lda + r] -= acc[i][jj][e];
            }
}

hipError_t launch_geqrf(const QrWork &w, hipStream_t s)
{
    for (int64_t j0 = 0; j0 < w.n; j0 += NB) {
        const int pw = (int)((w.n - j0) < NB ? (w.n - j0) : NB);
        const int64_t mk = w.m - j0;
        const PanelTree pt = panel_tree(mk);
        // 1. TSQR up the tree
        for (int l = 0; l < pt.levels; ++l)
            hipLaunchKernelGGL(tsqr_factor_kernel, dim3((unsigned)pt.nodes[l]), dim3(TS_NT), 0, s, w, j0, pw, l,
                               pt.nodes[l], l > 0 ? pt.nodes[l - 1] : 0, mk);
        // 2. explicit Q down the tree (level 0 lands in the panel)
        for (int l = pt.levels - 1; l >= 0; --l)
            hipLaunchKernelGGL(tsqr_formq_kernel, dim3((unsigned)pt.nodes[l]), dim3(TS_NT), 0, s, w, j0, pw, l,
                               pt.nodes[l], l == pt.levels - 1 ? 1 : 0, mk);
        // 3. Householder vectors, T, R and tau from the explicit Q
        hipLaunchKernelGGL(tsqr_lu_kernel, dim3(1), dim3(256), 0, s, w, j0, pw, pt.levels - 1);
        if (mk > pw)
            hipLaunchKernelGGL(tsqr_trsm_kernel, dim3((unsigned)((mk - pw + 255) / 256)), dim3(256), 0, s, w, j0,
                               pw);
        // 4. trailing update of the remaining columns (b included)
        const int64_t nt = w.ncols - j0 - pw;
        if (nt <= 0)
            continue;
        const int64_t ncb = (nt + WS::BN - 1) / WS::BN;
        int64_t nch = (2048 + ncb - 1) / ncb;
        if (nch > MAX_CHUNKS)
            nch = MAX_CHUNKS;
        int64_t chunk = (mk + nch - 1) / nch;
        chunk = (chunk + 15) & ~int64_t(15);
        if (chunk < 256)
            chunk = 256;
        nch = (mk + chunk - 1) / chunk;
        hipLaunchKernelGGL(qr_wpart_kernel, dim3((unsigned)ncb, (unsigned)nch), dim3(256), 0, s, w, j0, pw,
                           chunk, nt);
        hipLaunchKernelGGL(qr_wred_kernel, dim3((unsigned)((nt + NB - 1) / NB)), dim3(256), 0, s, w, pw, nch,
                           nt);
        hipLaunchKernelGGL(qr_update_kernel,
                           dim3((unsigned)((mk + US::BN - 1) / US::BN), (unsigned)((nt + US::BM - 1) / US::BM)),
                           dim3(256), 0, s, w, j0, pw, nt);
    }
    return hipGetLastError();
}

}  // namespace gap
