// CUR sparse-point selection (Sec. Implementation: sparse points chosen by
// CUR-based methods, after Mahoney & Drineas 2009).  For the n x d matrix X of
// descriptor rows, the leverage of row i over the row space of X is
//   lev_i = x_i^T (X^T X)^-1 x_i = ||x_i U^-1||^2,  X^T X = U^T U,
// and M rows are taken either as the M largest leverages or, with one Exp(1)
// variate e_i per row from the caller, as a sample without replacement with
// probabilities proportional to the leverage: the M smallest keys e_i / lev_i
// (the exponential-key method of Efraimidis & Spirakis).  Equal keys are taken
// in row order; the indices come out ascending.
//
// Steps: G = X^T X on FP64 MFMA (split over row chunks, upper block pairs,
// fixed-order sum), the Cholesky factor U (the K_MM factorisation), W = U^-1
// (one workgroup per column), Y = X W on FP64 MFMA with the row sums of squares
// in the epilogue (W upper triangular: a column tile needs k up to its last
// column only), keys, then the M-th smallest key by an 8-pass radix select on
// its bits and an ordered compaction.
#include <stddef.h>

#include "kernels.h"

namespace gap {

using CS = TileShape<128, 128, 16, 2, 2>;  // Gram blocks and projection tiles
constexpr int CUR_NB = 128;                // block of G / column tile of Y
constexpr int64_t CUR_MAX_CHUNKS = 64;     // row chunks of the Gram product
constexpr int CUR_SEL_NT = 256;
constexpr int CUR_SEL_PER = 4096;          // keys per workgroup in the compaction
constexpr int CUR_MAX_D = 4096;

struct CurState {
    unsigned long long prefix, mask;  // radix select: bits fixed so far
    long long k;                      // rank still to find among keys matching the prefix
    int32_t status;
    int32_t pad;
};

int64_t cur_nb(int d) { return (d + CUR_NB - 1) / CUR_NB; }
int64_t cur_chunks(int64_t n, int d)
{
    const int64_t nb = cur_nb(d), pairs = nb * (nb + 1) / 2;
    int64_t nch = (2048 + pairs - 1) / pairs;
    if (nch > CUR_MAX_CHUNKS)
        nch = CUR_MAX_CHUNKS;
    if (nch > (n + 255) / 256)
        nch = (n + 255) / 256;
    return nch < 1 ? 1 : nch;
}
int64_t cur_sel_blocks(int64_t n) { return (n + CUR_SEL_PER - 1) / CUR_SEL_PER; }

// Byte offsets of the workspace parts (each 256-aligned).
struct CurLayout {
    size_t state, G, part, W, rowpart, keys, hist, cnt, base, total;
};
CurLayout cur_layout(int64_t n, int d)
{
    CurLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = (o + bytes + 255) / 256 * 256;
        return at;
    };
    const int64_t nb = cur_nb(d), pairs = nb * (nb + 1) / 2;
    L.state = take(sizeof(CurState));
    L.G = take(sizeof(double) * (size_t)d * (size_t)d);
    L.part = take(sizeof(double) * (size_t)cur_chunks(n, d) * (size_t)pairs * CUR_NB * CUR_NB);
    L.W = take(sizeof(double) * (size_t)d * (size_t)d);
    L.rowpart = take(sizeof(double) * (size_t)nb * (size_t)n);
    L.keys = take(sizeof(double) * (size_t)n);
    L.hist = take(sizeof(unsigned) * 256);
    L.cnt = take(sizeof(long long) * 2 * (size_t)cur_sel_blocks(n));
    L.base = take(sizeof(long long) * 2 * (size_t)cur_sel_blocks(n));
    L.total = o;
    return L;
}

// Block pair index -> (bi, bj), bi <= bj, row-major over the upper triangle.
DEV void cur_pair(int64_t bp, int64_t nb, int64_t &bi, int64_t &bj)
{
    bi = 0;
    int64_t rem = bp;
    while (rem >= nb - bi) {
        rem -= nb - bi;
        ++bi;
    }
    bj = bi + rem;
}

// v = X[r][c0 .. c0 + LEN) (zero past the row's end or for r >= r_hi).
template <int LEN>
DEV void cur_row_run(const double *__restrict__ X, int64_t r, int64_t r_hi, int d, int64_t c0, bool even,
                     double (&v)[LEN])
{
    if (r < r_hi && even && c0 + LEN <= d) {
        load_run(X + r * d + c0, v);
    } else {
#pragma unroll
        for (int e = 0; e < LEN; ++e)
            v[e] = (r < r_hi && c0 + e < d) ? X[r * d + c0 + e] : 0.0;
    }
}

// Partial Gram block (bi, bj) over the rows of chunk blockIdx.y:
// part[ch][bp][p][q] = sum_r X[r][128 bi + p] X[r][128 bj + q].
__global__ __launch_bounds__(256, 2) void cur_gram_kernel(const double *__restrict__ X, int64_t n, int d,
                                                          int64_t nb, int64_t chunk, double *__restrict__ part)
{
    __shared__ double lds[2 * CS::STAGE];
    const int64_t bp = blockIdx.x, ch = blockIdx.y, pairs = gridDim.x;
    int64_t bi, bj;
    cur_pair(bp, nb, bi, bj);
    const int64_t p0 = bi * CUR_NB, q0 = bj * CUR_NB;
    const int64_t rlo = ch * chunk;
    const int64_t rhi = (rlo + chunk) < n ? (rlo + chunk) : n;
    d4 acc[CS::FM][CS::FN];
    zero_acc<CS>(acc);
    if (rlo < rhi) {
        constexpr int VA = CS::BM * CS::BK / CS::NT, VB = CS::BN * CS::BK / CS::NT;
        const bool even = (d & 1) == 0;
        // runs along the descriptor index (contiguous in a row of X)
        auto fa = [&](int p, int64_t k, double (&v)[VA]) { cur_row_run<VA>(X, rlo + k, rhi, d, p0 + p, even, v); };
        auto fb = [&](int q, int64_t k, double (&v)[VB]) { cur_row_run<VB>(X, rlo + k, rhi, d, q0 + q, even, v); };
        gemm_tile_runs<CS, false, false>(acc, lds, rhi - rlo, fa, fb);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / CS::WN, wn = wave % CS::WN;
    double *P = part + (ch * pairs + bp) * (int64_t)(CUR_NB * CUR_NB);
#pragma unroll
    for (int i = 0; i < CS::FM; ++i)
#pragma unroll
        for (int j = 0; j < CS::FN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                P[acc_row<CS>(wm, i, lane, e) * CUR_NB + acc_col<CS>(wn, j, lane, e)] = acc[i][j][e];
}

// G (column-major, leading dimension d, both triangles) from the partials, the
// chunks summed in order.  One element of one block pair per thread.
__global__ __launch_bounds__(256) void cur_gram_sum_kernel(const double *__restrict__ part, int64_t nch,
                                                           int64_t pairs, int64_t nb, int d, double *__restrict__ G)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= pairs * CUR_NB * CUR_NB)
        return;
    const int64_t bp = e / (CUR_NB * CUR_NB), pq = e % (CUR_NB * CUR_NB);
    int64_t bi, bj;
    cur_pair(bp, nb, bi, bj);
    const int64_t p = bi * CUR_NB + pq / CUR_NB, q = bj * CUR_NB + pq % CUR_NB;
    if (p >= d || q >= d)
        return;
    double s = 0.0;
    for (int64_t ch = 0; ch < nch; ++ch)
        s += part[(ch * pairs + bp) * (int64_t)(CUR_NB * CUR_NB) + pq];
    G[q * d + p] = s;
    G[p * d + q] = s;
}

// W = U^-1 for the upper triangular U (column-major, leading dimension d):
// workgroup j solves U w = e_j by back substitution, right-looking (w_i from
// b_i, then b_k -= U[k][i] w_i for k < i), and writes column j of W.
__global__ __launch_bounds__(256) void cur_trinv_kernel(const double *__restrict__ U, int d, double *__restrict__ W)
{
    __shared__ double b[CUR_MAX_D];
    __shared__ double wi_s;
    const int j = blockIdx.x, t = threadIdx.x;
    for (int k = t; k < d; k += 256)
        b[k] = (k == j) ? 1.0 : 0.0;
    for (int i = t + j + 1; i < d; i += 256)
        W[(int64_t)j * d + i] = 0.0;
    for (int i = j; i >= 0; --i) {
        __syncthreads();
        if (t == 0) {
            wi_s = b[i] / U[(int64_t)i * d + i];
            W[(int64_t)j * d + i] = wi_s;
        }
        __syncthreads();
        const double wi = wi_s;
        const double *Ui = U + (int64_t)i * d;
        for (int k = t; k < i; k += 256)
            b[k] -= Ui[k] * wi;
    }
}

// Y = X W for the rows of tile blockIdx.x and the 128 columns of tile
// blockIdx.y; rowpart[ct][r] = sum over the tile's columns of Y[r][q]^2, the
// columns summed in order.
__global__ __launch_bounds__(256, 2) void cur_proj_kernel(const double *__restrict__ X, int64_t n, int d,
                                                          const double *__restrict__ W, double *__restrict__ rowpart)
{
    __shared__ double lds[2 * CS::STAGE];
    const int64_t r0 = (int64_t)blockIdx.x * CS::BM, ct = blockIdx.y, q0 = ct * CUR_NB;
    const int64_t K = (q0 + CUR_NB) < d ? (q0 + CUR_NB) : d;  // W[k][q] = 0 for k > q
    d4 acc[CS::FM][CS::FN];
    zero_acc<CS>(acc);
    constexpr int VA = CS::BM * CS::BK / CS::NT, VB = CS::BN * CS::BK / CS::NT;
    const bool even = (d & 1) == 0;
    auto fa = [&](int r, int64_t k, double (&v)[VA]) {  // X[r0 + r][k .. k + VA)
        const int64_t row = r0 + r;
        if (row < n && even && k + VA <= K) {
            load_run(X + row * d + k, v);
        } else {
#pragma unroll
            for (int e = 0; e < VA; ++e)
                v[e] = (row < n && k + e < K) ? X[row * d + k + e] : 0.0;
        }
    };
    auto fb = [&](int q, int64_t k, double (&v)[VB]) {  // W[k .. k + VB)[q0 + q], contiguous along k
        const int64_t col = q0 + q;
        if (col < d && even && k + VB <= K) {
            load_run(W + col * d + k, v);
        } else {
#pragma unroll
            for (int e = 0; e < VB; ++e)
                v[e] = (col < d && k + e < K) ? W[col * d + k + e] : 0.0;
        }
    };
    gemm_tile_runs<CS, true, true>(acc, lds, K, fa, fb);
    // squares parked 64 columns at a time (the columns of waves wn = h), then
    // thread r < 128 sums row r over them in column order
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave / CS::WN, wn = wave % CS::WN;
    double *E = lds;  // [128][65]
    double rs = 0.0;
    for (int h = 0; h < CS::WN; ++h) {
        if (wn == h) {
#pragma unroll
            for (int i = 0; i < CS::FM; ++i)
#pragma unroll
                for (int j = 0; j < CS::FN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int rr = acc_row<CS>(wm, i, lane, e), cc = acc_col<CS>(wn, j, lane, e) - h * CS::TN;
                        E[rr * (CS::TN + 1) + cc] = acc[i][j][e] * acc[i][j][e];
                    }
        }
        __syncthreads();
        if (t < CS::BM)
            for (int c = 0; c < CS::TN; ++c)
                rs += E[t * (CS::TN + 1) + c];
        __syncthreads();
    }
    if (t < CS::BM && r0 + t < n)
        rowpart[ct * n + r0 + t] = rs;
}

// lev = sum of the column tiles' parts in order; key = draw / lev (1 / lev
// without draws), +inf for a zero row.
__global__ __launch_bounds__(256) void cur_keys_kernel(const double *__restrict__ rowpart, int64_t n, int64_t nct,
                                                       const double *__restrict__ draws, double *__restrict__ lev_out,
                                                       double *__restrict__ keys)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    double l = 0.0;
    for (int64_t ct = 0; ct < nct; ++ct)
        l += rowpart[ct * n + i];
    if (lev_out)
        lev_out[i] = l;
    double k = (draws ? draws[i] : 1.0) / l;
    if (!(k == k))
        k = __builtin_inf();
    keys[i] = k;
}

__global__ void cur_select_init_kernel(CurState *st, unsigned *hist, long long M)
{
    const int t = threadIdx.x;
    if (t < 256)
        hist[t] = 0u;
    if (t == 0) {
        st->prefix = 0ull;
        st->mask = 0ull;
        st->k = M;
        st->status = 0;
    }
}

// Histogram of bits [shift, shift + 8) of the keys whose higher bits match the prefix.
__global__ __launch_bounds__(256) void cur_hist_kernel(const double *__restrict__ keys, int64_t n,
                                                       const CurState *__restrict__ st, int shift,
                                                       unsigned *__restrict__ hist)
{
    __shared__ unsigned h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const unsigned long long prefix = st->prefix, mask = st->mask;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(keys[i]);
        if ((b & mask) == prefix)
            atomicAdd(&h[(b >> shift) & 255ull], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x])
        atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Fix the next 8 bits: the digit whose cumulative count first reaches k.
__global__ __launch_bounds__(256) void cur_pick_kernel(CurState *st, unsigned *hist, int shift)
{
    __shared__ long long c[256];
    const int t = threadIdx.x;
    c[t] = hist[t];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const long long v = t >= off ? c[t - off] : 0;
        __syncthreads();
        c[t] += v;
        __syncthreads();
    }
    const long long k = st->k;
    const long long below = t > 0 ? c[t - 1] : 0;
    __syncthreads();
    if (below < k && c[t] >= k) {
        st->k = k - below;
        st->prefix |= (unsigned long long)t << shift;
        st->mask |= 255ull << shift;
    }
    hist[t] = 0u;
}

// Per compaction block: keys below the threshold T and keys equal to it.
__global__ __launch_bounds__(CUR_SEL_NT) void cur_count_kernel(const double *__restrict__ keys, int64_t n,
                                                               const CurState *__restrict__ st,
                                                               long long *__restrict__ cnt)
{
    __shared__ long long sl[CUR_SEL_NT], se[CUR_SEL_NT];
    const unsigned long long T = st->prefix;
    const int64_t lo = (int64_t)blockIdx.x * CUR_SEL_PER;
    const int64_t hi = (lo + CUR_SEL_PER) < n ? (lo + CUR_SEL_PER) : n;
    long long a = 0, b = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += CUR_SEL_NT) {
        const unsigned long long x = (unsigned long long)__double_as_longlong(keys[i]);
        a += x < T;
        b += x == T;
    }
    sl[threadIdx.x] = a;
    se[threadIdx.x] = b;
    __syncthreads();
    for (int off = CUR_SEL_NT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sl[threadIdx.x] += sl[threadIdx.x + off];
            se[threadIdx.x] += se[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cnt[2 * blockIdx.x] = sl[0];
        cnt[2 * blockIdx.x + 1] = se[0];
    }
}

// Exclusive prefix sums of the per-block counts (one workgroup).
__global__ __launch_bounds__(256) void cur_scan_kernel(const long long *__restrict__ cnt, int64_t nblk,
                                                       long long *__restrict__ base)
{
    __shared__ long long carry_l, carry_e;
    __shared__ long long sl[256], se[256];
    const int t = threadIdx.x;
    if (t == 0) {
        carry_l = 0;
        carry_e = 0;
    }
    __syncthreads();
    for (int64_t b0 = 0; b0 < nblk; b0 += 256) {
        const int64_t b = b0 + t;
        const long long l = b < nblk ? cnt[2 * b] : 0, e = b < nblk ? cnt[2 * b + 1] : 0;
        sl[t] = l;
        se[t] = e;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const long long vl = t >= off ? sl[t - off] : 0, ve = t >= off ? se[t - off] : 0;
            __syncthreads();
            sl[t] += vl;
            se[t] += ve;
            __syncthreads();
        }
        if (b < nblk) {
            base[2 * b] = carry_l + sl[t] - l;
            base[2 * b + 1] = carry_e + se[t] - e;
        }
        __syncthreads();
        if (t == 255) {
            carry_l += sl[255];
            carry_e += se[255];
        }
        __syncthreads();
    }
}

// Write the selected row indices in ascending order: row i is taken when its
// key is below T, or equal to T and among the first k such rows; its place is
// (rows taken before it) = less_before + min(equal_before, k).
__global__ __launch_bounds__(CUR_SEL_NT) void cur_write_kernel(const double *__restrict__ keys, int64_t n,
                                                               const CurState *__restrict__ st,
                                                               const long long *__restrict__ base,
                                                               int64_t *__restrict__ out)
{
    __shared__ int sl[CUR_SEL_NT], se[CUR_SEL_NT];
    __shared__ long long run_l, run_e;
    const unsigned long long T = st->prefix;
    const long long kq = st->k;
    const int t = threadIdx.x;
    const int64_t lo = (int64_t)blockIdx.x * CUR_SEL_PER;
    const int64_t hi = (lo + CUR_SEL_PER) < n ? (lo + CUR_SEL_PER) : n;
    if (t == 0) {
        run_l = base[2 * blockIdx.x];
        run_e = base[2 * blockIdx.x + 1];
    }
    __syncthreads();
    for (int64_t i0 = lo; i0 < hi; i0 += CUR_SEL_NT) {
        const int64_t i = i0 + t;
        int fl = 0, fe = 0;
        if (i < hi) {
            const unsigned long long x = (unsigned long long)__double_as_longlong(keys[i]);
            fl = x < T;
            fe = x == T;
        }
        sl[t] = fl;
        se[t] = fe;
        __syncthreads();
        for (int off = 1; off < CUR_SEL_NT; off <<= 1) {
            const int vl = t >= off ? sl[t - off] : 0, ve = t >= off ? se[t - off] : 0;
            __syncthreads();
            sl[t] += vl;
            se[t] += ve;
            __syncthreads();
        }
        const long long lb = run_l + sl[t] - fl, eb = run_e + se[t] - fe;  // before row i
        if (fl || (fe && eb < kq))
            out[lb + (eb < kq ? eb : kq)] = i;
        __syncthreads();
        if (t == CUR_SEL_NT - 1) {
            run_l += sl[t];
            run_e += se[t];
        }
        __syncthreads();
    }
}

size_t cur_workspace_bytes(int64_t n, int d) { return cur_layout(n, d).total; }
size_t cur_status_offset() { return offsetof(CurState, status); }

hipError_t launch_cur_select(const CurLaunch &c, hipStream_t s)
{
    const int64_t n = c.n;
    const int d = c.d;
    const CurLayout L = cur_layout(n, d);
    char *ws = static_cast<char *>(c.workspace);
    CurState *st = reinterpret_cast<CurState *>(ws + L.state);
    double *G = reinterpret_cast<double *>(ws + L.G);
    double *part = reinterpret_cast<double *>(ws + L.part);
    double *W = reinterpret_cast<double *>(ws + L.W);
    double *rowpart = reinterpret_cast<double *>(ws + L.rowpart);
    double *keys = reinterpret_cast<double *>(ws + L.keys);
    unsigned *hist = reinterpret_cast<unsigned *>(ws + L.hist);
    long long *cnt = reinterpret_cast<long long *>(ws + L.cnt);
    long long *base = reinterpret_cast<long long *>(ws + L.base);
    const int64_t nb = cur_nb(d), pairs = nb * (nb + 1) / 2, nch = cur_chunks(n, d);
    int64_t chunk = (n + nch - 1) / nch;
    chunk = (chunk + 15) / 16 * 16;
    hipLaunchKernelGGL(cur_select_init_kernel, dim3(1), dim3(256), 0, s, st, hist, (long long)c.M);
    hipLaunchKernelGGL(cur_gram_kernel, dim3((unsigned)pairs, (unsigned)nch), dim3(256), 0, s, c.x, n, d, nb, chunk,
                       part);
    hipLaunchKernelGGL(cur_gram_sum_kernel, dim3((unsigned)((pairs * CUR_NB * CUR_NB + 255) / 256)), dim3(256), 0, s,
                       part, nch, pairs, nb, d, G);
    hipError_t e = launch_potrf_upper(G, d, d, &st->status, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(cur_trinv_kernel, dim3((unsigned)d), dim3(256), 0, s, G, d, W);
    hipLaunchKernelGGL(cur_proj_kernel, dim3((unsigned)((n + CS::BM - 1) / CS::BM), (unsigned)nb), dim3(256), 0, s,
                       c.x, n, d, W, rowpart);
    hipLaunchKernelGGL(cur_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rowpart, n, nb, c.draws,
                       c.lev_out, keys);
    int64_t hg = (n + 255) / 256;
    if (hg > 2048)
        hg = 2048;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 56 - 8 * pass;
        hipLaunchKernelGGL(cur_hist_kernel, dim3((unsigned)hg), dim3(256), 0, s, keys, n, st, shift, hist);
        hipLaunchKernelGGL(cur_pick_kernel, dim3(1), dim3(256), 0, s, st, hist, shift);
    }
    const int64_t nblk = cur_sel_blocks(n);
    hipLaunchKernelGGL(cur_count_kernel, dim3((unsigned)nblk), dim3(CUR_SEL_NT), 0, s, keys, n, st, cnt);
    hipLaunchKernelGGL(cur_scan_kernel, dim3(1), dim3(256), 0, s, cnt, nblk, base);
    hipLaunchKernelGGL(cur_write_kernel, dim3((unsigned)nblk), dim3(CUR_SEL_NT), 0, s, keys, n, st, base, c.out);
    return hipGetLastError();
}

int cur_max_d() { return CUR_MAX_D; }

}  // namespace gap
