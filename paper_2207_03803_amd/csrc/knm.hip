// K_NM / K_MM builder: descriptor GEMM on FP64 MFMA with the dot-product
// covariance, the per-configuration segment-sum and the Sigma^-1/2 row scale
// fused into the epilogue (Sec. Theory: definition of K_MN; the upper block of
// A; Eqs. 1-2).  The n_atoms x M matrix of atom-level covariances is never
// written to HBM.
#include "knm.h"

namespace gap {

// ---------------------------------------------------------------------------
// Tile plan.  The rows of K_NM are independent per configuration, so a tile
// may hold any set of whole configurations.  The configurations are split, in
// order, into chunks of PLAN_C; each chunk is sorted by atom count (largest
// first, then by index) and packed by one thread: a configuration of more than
// KNM_CAP atoms gets a tile of its own (processed in atom chunks); the others
// fill tiles of at most KNM_CAP atoms and KNM_MAX_SEG configurations, each
// tile taking the largest remaining configuration that still fits until none
// does.  Output: cfg_list (the configurations, tile by tile) and tile_start[t]
// (the first position of tile t in cfg_list).  The offsets are validated too.
// ---------------------------------------------------------------------------
constexpr int PLAN_C = 2048;               // configurations per chunk
constexpr int PLAN_LARGE = KNM_CAP + 1;    // bucket of the configurations above KNM_CAP atoms
constexpr int PLAN_WORDS = (PLAN_LARGE + 64) / 64;

int64_t knm_plan_chunks(int64_t N) { return (N + PLAN_C - 1) / PLAN_C; }

__global__ __launch_bounds__(256) void plan_chunk_kernel(const int64_t *__restrict__ offsets, int64_t N,
                                                         int64_t n_atoms, int32_t *__restrict__ cfg_list,
                                                         int32_t *__restrict__ lstart, int32_t *__restrict__ lcount,
                                                         int32_t *status)
{
    __shared__ int64_t key[PLAN_C];
    __shared__ int32_t bfirst[PLAN_LARGE + 1], blast[PLAN_LARGE + 1];
    __shared__ int bad_s;
    const int t = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * PLAN_C;
    const int cnt = (int)((N - c0) < PLAN_C ? (N - c0) : PLAN_C);
    if (t == 0) {
        bad_s = 0;
        if (blockIdx.x == 0 && offsets[0] != 0)
            bad_s = 1;
        if (c0 + cnt == N && offsets[N] != n_atoms)
            bad_s = 1;
    }
    for (int b = t; b <= PLAN_LARGE; b += 256)
        bfirst[b] = blast[b] = 0;
    __syncthreads();
    // key = (PLAN_LARGE - bucket) << 32 | local index: ascending = largest first
    for (int i = t; i < PLAN_C; i += 256) {
        int64_t k = INT64_MAX;
        if (i < cnt) {
            const int64_t sz = offsets[c0 + i + 1] - offsets[c0 + i];
            if (sz < 0)
                bad_s = 1;
            const int64_t b = sz > KNM_CAP ? PLAN_LARGE : (sz < 0 ? 0 : sz);
            k = ((int64_t)(PLAN_LARGE - b) << 32) | i;
        }
        key[i] = k;
    }
    __syncthreads();
    for (int kk = 2; kk <= PLAN_C; kk <<= 1)
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int i = t; i < PLAN_C; i += 256) {
                const int l = i ^ jj;
                if (l > i) {
                    const int64_t x = key[i], y = key[l];
                    if ((x > y) == ((i & kk) == 0)) {
                        key[i] = y;
                        key[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    // bucket b occupies sorted positions [bfirst[b], blast[b])
    for (int i = t; i < cnt; i += 256) {
        const int b = PLAN_LARGE - (int)(key[i] >> 32);
        if (i == 0 || (key[i - 1] >> 32) != (key[i] >> 32))
            bfirst[b] = i;
        if (i == cnt - 1 || (key[i + 1] >> 32) != (key[i] >> 32))
            blast[b] = i + 1;
    }
    __syncthreads();
    if (t != 0)
        return;
    int32_t *ls = lstart + blockIdx.x * (int64_t)(PLAN_C + 1);
    if (bad_s) {
        set_status(status, DST_EINVAL);
        lcount[blockIdx.x] = 0;
        return;
    }
    int pos = 0, ntile = 0;
    for (int i = bfirst[PLAN_LARGE]; i < blast[PLAN_LARGE]; ++i) {  // one tile each
        ls[ntile++] = pos;
        cfg_list[c0 + pos++] = (int32_t)(c0 + (key[i] & 0xffffffff));
    }
    // non-empty buckets 0..KNM_CAP as a bit set; bfirst[] is each bucket's next item
    uint64_t nonempty[PLAN_WORDS];
    for (int w = 0; w < PLAN_WORDS; ++w)
        nonempty[w] = 0;
    for (int b = 0; b <= KNM_CAP; ++b)
        if (bfirst[b] < blast[b])
            nonempty[b >> 6] |= 1ull << (b & 63);
    while (pos < cnt) {
        ls[ntile++] = pos;
        int r = KNM_CAP, nseg = 0;
        while (nseg < KNM_MAX_SEG) {
            // largest non-empty bucket b <= r
            int found = -1;
            for (int w = r >> 6; w >= 0 && found < 0; --w) {
                uint64_t m = nonempty[w];
                if (w == (r >> 6))
                    m &= ((r & 63) == 63) ? ~0ull : ((1ull << ((r & 63) + 1)) - 1);
                if (m)
                    found = w * 64 + 63 - __clzll(m);
            }
            if (found < 0)
                break;
            const int i = bfirst[found]++;
            if (bfirst[found] == blast[found])
                nonempty[found >> 6] &= ~(1ull << (found & 63));
            cfg_list[c0 + pos++] = (int32_t)(c0 + (key[i] & 0xffffffff));
            r -= found;
            ++nseg;
        }
    }
    lcount[blockIdx.x] = ntile;
}

// Global tile table: tile_start[base_c + j] = chunk c's j-th tile, n_tiles.
__global__ __launch_bounds__(256) void plan_publish_kernel(const int32_t *__restrict__ lstart,
                                                           const int32_t *__restrict__ lcount, int64_t n_chunks,
                                                           int64_t N, int32_t *__restrict__ tile_start,
                                                           int32_t *__restrict__ n_tiles, int64_t max_tiles,
                                                           int32_t *status)
{
    __shared__ int64_t base_s;
    const int64_t c = blockIdx.x;
    if (threadIdx.x == 0) {
        int64_t b = 0;
        for (int64_t q = 0; q < c; ++q)
            b += lcount[q];
        base_s = b;
    }
    __syncthreads();
    const int64_t base = base_s, nt = lcount[c];
    const bool bad = (*status != 0) || base + nt > max_tiles;
    if (!bad)
        for (int64_t j = threadIdx.x; j < nt; j += 256)
            tile_start[base + j] = (int32_t)(c * PLAN_C + lstart[c * (PLAN_C + 1) + j]);
    if (c == n_chunks - 1 && threadIdx.x == 0) {
        if (bad) {
            if (base + nt > max_tiles)
                set_status(status, DST_EINVAL);
            *n_tiles = 0;
        } else {
            tile_start[base + nt] = (int32_t)N;
            *n_tiles = (int32_t)(base + nt);
        }
    }
}

int64_t knm_max_tiles(int64_t N, int64_t n_atoms)
{
    // Within a chunk, a tile closes only when the largest remaining
    // configuration does not fit, so two consecutive tiles hold more than
    // KNM_CAP atoms unless the first was closed by the configuration cap; each
    // chunk may end with one more partial tile.
    int64_t bound = 2 * ((n_atoms + KNM_CAP - 1) / KNM_CAP) + (N + KNM_MAX_SEG - 1) / KNM_MAX_SEG +
                    knm_plan_chunks(N) + 1;
    return bound < N ? bound : N;
}

// 256 threads, 4 waves of 64 x BN (BN = 64 by default, 32 as a tuning choice),
// BK = 8: two workgroups share a CU and cover each other's barriers.
template <int BN>
using KSB = TileShape<KNM_BM, BN, 8, 4, 1>;
using KS = KSB<KNM_BN>;
static_assert(KS::NT == 256, "K_NM kernel assumes 256 threads");
static_assert(!KS::M16, "the predict row sums assume the 4x4x4 accumulator layout");
static_assert(KNM_BM == 256 && KNM_BN == 64, "loader mapping assumes 256-atom tiles");

constexpr int EPC = 32;           // epilogue columns per pass (two 16-column blocks)
constexpr int EPLD = EPC + 1;     // padded LDS row of the epilogue buffer

// Load one BK-slice (8 descriptor components) of the atom tile (256 rows) and
// the sparse tile (BN rows) into registers.  Rows past the valid range and k
// past d read as zero.  Each thread loads 8 k of its atom row and BN / 32 k of
// sparse row tid / (256 / BN).
template <int BN>
struct KnmLoads {
    double a[8];
    double b[BN / 32];
    bool za = false, zb = false;  // store zeros instead (a missing row, see knm_load_full)
};

template <int BN>
DEV void knm_load(KnmLoads<BN> &r, const double *__restrict__ xr, const double *__restrict__ XM, int64_t col0,
                  int64_t M, int d, int k0)
{
    constexpr int TPR = 256 / BN, VB = BN / 32;  // threads per sparse row, k per thread
    const int tid = threadIdx.x;
    {
        // xr: this thread's atom row (nullptr past the tile's atoms)
        const int kb = k0;
        if (xr && kb + 8 <= d) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                r.a[e] = xr[kb + e];
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                r.a[e] = (xr && kb + e < d) ? xr[kb + e] : 0.0;
        }
    }
    {
        const int64_t row = col0 + tid / TPR;
        const int kb = k0 + (tid % TPR) * VB;
        const bool rv = row < M;
        const double *p = XM + row * (int64_t)d + kb;
        if (rv && kb + VB <= d) {
#pragma unroll
            for (int e = 0; e < VB; ++e)
                r.b[e] = p[e];
        } else {
#pragma unroll
            for (int e = 0; e < VB; ++e)
                r.b[e] = (rv && kb + e < d) ? p[e] : 0.0;
        }
    }
}

// The same for a slice that lies inside the rows (k0 + 8 <= d), without
// branches: a thread whose atom or sparse row is missing reads row 0 of XM
// instead and stores zeros, so the loads stay in flight through the stage's
// MFMAs (a divergent branch here makes the compiler wait for them before).
template <int BN>
DEV void knm_load_full(KnmLoads<BN> &r, const double *__restrict__ xr, const double *__restrict__ XM,
                       int64_t col0, int64_t M, int d, int k0)
{
    constexpr int TPR = 256 / BN, VB = BN / 32;
    const int tid = threadIdx.x;
    r.za = !xr;
    const double *sa = xr ? xr + k0 : XM + k0;
#pragma unroll
    for (int e = 0; e < 8; ++e)
        r.a[e] = sa[e];
    const int64_t row = col0 + tid / TPR;
    const int kb = k0 + (tid % TPR) * VB;
    r.zb = row >= M;
    const double *sb = row < M ? XM + row * (int64_t)d + kb : XM + kb;
#pragma unroll
    for (int e = 0; e < VB; ++e)
        r.b[e] = sb[e];
}

template <int BN>
DEV void knm_store(const KnmLoads<BN> &r, double *As, double *Bs)
{
    using S = KSB<BN>;
    constexpr int TPR = 256 / BN, VB = BN / 32;
    const int tid = threadIdx.x;
    {
        const int row = tid;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            As[e * S::LDA + row] = r.za ? 0.0 : r.a[e];
    }
    {
        const int row = tid / TPR, kb = (tid % TPR) * VB;
#pragma unroll
        for (int e = 0; e < VB; ++e)
            Bs[(kb + e) * S::LDB + row] = r.zb ? 0.0 : r.b[e];
    }
}

// G = (the tile's 256 atom rows, thread t's row at xr) . XM[col0 : col0+BN)^T,
// accumulated in registers.
template <int BN>
DEV void knm_gemm(d4 (&acc)[KSB<BN>::FM][KSB<BN>::FN], double *lds, const double *__restrict__ xr,
                  const double *__restrict__ XM, int64_t col0, int64_t M, int d)
{
    using S = KSB<BN>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / S::WN, wn = wave % S::WN;
    zero_acc<S>(acc);
    const int nk = (d + S::BK - 1) / S::BK;
    const int nkf = d / S::BK;  // slices inside the rows; a ragged last one is loaded with checks
    KnmLoads<BN> r;
    if (nkf > 0)
        knm_load_full<BN>(r, xr, XM, col0, M, d, 0);
    else
        knm_load<BN>(r, xr, XM, col0, M, d, 0);
    knm_store<BN>(r, lds, lds + S::A_ELEMS);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        double *cur = lds + (kt & 1) * S::STAGE;
        double *nxt = lds + ((kt + 1) & 1) * S::STAGE;
        const bool more = kt + 1 < nkf;
        if (more)
            knm_load_full<BN>(r, xr, XM, col0, M, d, (kt + 1) * S::BK);
        mma_stage<S>(cur, cur + S::A_ELEMS, acc, wm, wn, lane);
        if (more) {
            knm_store<BN>(r, nxt, nxt + S::A_ELEMS);
        } else if (kt + 1 < nk) {  // the ragged last slice, loaded after this stage's MFMAs
            knm_load<BN>(r, xr, XM, col0, M, d, (kt + 1) * S::BK);
            knm_store<BN>(r, nxt, nxt + S::A_ELEMS);
        }
        __syncthreads();
    }
}

template <int BN>
constexpr int knm_lds_doubles()
{
    return (2 * KSB<BN>::STAGE > KNM_BM * EPLD) ? 2 * KSB<BN>::STAGE : KNM_BM * EPLD;
}

// One workgroup's tile; bid = the workgroup's index within this K_NM's own grid
// (a multiple-of-8 offset into a grouped grid keeps bid's XCD the hardware's).
// A derivative position whose gradient row and atom are in range.
DEV bool kdm_valid(const KnmArgs &a, int64_t pos)
{
    const int64_t g = a.pos_grad[pos];
    return g >= 0 && g < a.n_grad && a.grad_atom[g] >= 0 && a.grad_atom[g] < a.n_src;
}

template <int BN, bool DERIV = false>
DEV void knm_body(const KnmArgs &a, int64_t bid)
{
    using KS = KSB<BN>;
    constexpr int KNM_BN = BN;
    static_assert(BN == 32 || BN == 64, "column tile of 32 or 64 sparse points");
    __shared__ double lds[knm_lds_doubles<BN>()];
    __shared__ int32_t sstart[KNM_MAX_SEG + 1];  // atom offset of each segment within the tile
    __shared__ int64_t sbase[KNM_MAX_SEG];       // first atom (row of X) of each segment
    __shared__ int32_t srow[KNM_MAX_SEG];        // output row of each segment
    __shared__ double carry[KNM_BN];
    __shared__ double rowf[DERIV ? KNM_BM : 1];      // derivative rows: zeta sw2 w of tile row r
    __shared__ int64_t rowatom[DERIV ? KNM_BM : 1];  // and its gradient's atom (-1 past the tile)

    // The grid is sized for the largest possible tile count; the remap uses
    // the actual count so that all eight XCDs get an equal share of the tiles.
    const bool unit = (a.offsets == nullptr);
    const int64_t n_tiles = unit ? (a.n_rows_unit + KNM_BM - 1) / KNM_BM : (int64_t)*a.n_tiles_dev;
    int64_t t, ct;
    if constexpr (DERIV) {
        // tiles dealt to the XCDs in turn (tile t to XCD t mod 8), each tile's column
        // tiles on its XCD in order: observations of very different sizes (multi-chunk
        // virials beside small force components) spread evenly over the XCDs
        const int64_t tiles8 = (n_tiles + 7) / 8;
        if (bid >= tiles8 * 8 * a.n_ct)
            return;
        const int64_t x = bid & 7, q = bid >> 3;
        t = 8 * (q / a.n_ct) + x;
        ct = q % a.n_ct;
        if (t >= n_tiles)
            return;
    } else {
        const int64_t total = n_tiles * a.n_ct;
        const int64_t total_pad = (total + 7) & ~int64_t(7);
        if (bid >= total_pad)
            return;
        const int64_t lw = xcd_remap(bid, total_pad);
        if (lw >= total)
            return;
        t = lw / a.n_ct;
        ct = lw % a.n_ct;
    }
    const int64_t col0 = ct * KNM_BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / KS::WN, wn = wave % KS::WN;

    // K_MM, upper triangle only: a tile wholly below the diagonal is zero (no product)
    if (unit && a.upper_only && t * KNM_BM > col0 + KNM_BN - 1) {
        const int64_t r0 = t * KNM_BM;
        const int nr = (int)((a.n_rows_unit - r0) < KNM_BM ? (a.n_rows_unit - r0) : KNM_BM);
        for (int item = tid; item < nr * KNM_BN; item += KS::NT) {
            const int r = item % nr, c = item / nr;
            const int64_t colg = col0 + c;
            if (colg < a.M)
                a.out[colg * a.ldo + a.row_off + r0 + r] = 0.0;
        }
        return;
    }

    // The tile's segments: rows of the unit block, or configurations from the plan.
    int n_seg;
    int64_t n_at;  // atoms in the tile
    if (unit) {
        const int64_t r0 = t * KNM_BM;
        n_seg = (int)((a.n_rows_unit - r0) < KNM_BM ? (a.n_rows_unit - r0) : KNM_BM);
        if (tid == 0)
            sstart[0] = 0;
        if (tid < n_seg) {
            sstart[tid + 1] = tid + 1;
            sbase[tid] = r0 + tid;
            srow[tid] = (int32_t)(r0 + tid);
        }
        n_at = n_seg;
    } else {
        const int64_t p0 = a.tile_start[t];
        n_seg = (int)(a.tile_start[t + 1] - p0);
        int64_t sz = 0;
        if (tid < n_seg) {
            const int32_t cfg = a.cfg_list[p0 + tid];
            const int64_t lo = a.offsets[cfg];
            sz = a.offsets[cfg + 1] - lo;
            sbase[tid] = lo;
            srow[tid] = cfg;
        }
        // inclusive scan of the segment sizes (one per thread)
        int32_t *scan = reinterpret_cast<int32_t *>(lds);
        scan[tid] = (int32_t)sz;
        __syncthreads();
        for (int off = 1; off < KNM_MAX_SEG; off <<= 1) {
            const int32_t x = (tid >= off) ? scan[tid - off] : 0;
            __syncthreads();
            scan[tid] += x;
            __syncthreads();
        }
        sstart[tid + 1] = scan[tid];
        if (tid == 0)
            sstart[0] = 0;
        __syncthreads();
        n_at = sstart[n_seg];
    }
    __syncthreads();

    // Row scale of segment s (loaded where its latency can overlap other work).
    auto sig = [&](int s) { return a.sigma ? a.sigma[srow[s]] : 1.0; };
    auto emit = [&](int s, int64_t colg, double sum, double sg) {
        const int64_t row = srow[s];
        double v = sum;
        if (unit) {
            if (row == colg)
                v += a.jitter;
            if (a.upper_only && row > colg)
                v = 0.0;
        }
        if (a.sigma)
            v = v / sg;
        a.out[colg * a.ldo + a.row_off + row] = v;
    };

    if (n_at == 0) {  // only empty configurations: their sums are zero
        for (int item = tid; item < n_seg * KNM_BN; item += KS::NT) {
            const int s = item % n_seg, c = item / n_seg;
            const int64_t colg = col0 + c;
            if (colg < a.M)
                emit(s, colg, 0.0, sig(s));
        }
        return;
    }

    // This thread's atom row for a tile of whole segments: segment by binary search.
    const double *xr_packed = nullptr;
    const bool multi = n_at > KNM_BM;  // then n_seg == 1: a configuration in several atom chunks
    if (!multi && tid < n_at) {
        int lo = 0, hi = n_seg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sstart[mid] <= tid)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int64_t pos = sbase[lo] + (tid - sstart[lo]);
        xr_packed = a.X + (DERIV ? a.pos_grad[pos] : pos) * (int64_t)a.d;
        if (DERIV && !kdm_valid(a, pos)) {
            xr_packed = nullptr;
            set_status(a.status, DST_EINVAL);
        }
    }
    d4 acc[KS::FM][KS::FN];
    for (int64_t cs = 0; cs < n_at; cs += KNM_BM) {
        const bool first = (cs == 0), last = (cs + KNM_BM >= n_at);
        const double *xr = xr_packed;
        if (multi) {
            const int64_t pos = sbase[0] + cs + tid;
            xr = (cs + tid < n_at) ? a.X + (DERIV ? a.pos_grad[pos] : pos) * (int64_t)a.d : nullptr;
            if (DERIV && xr && !kdm_valid(a, pos)) {
                xr = nullptr;
                set_status(a.status, DST_EINVAL);
            }
        }
        if constexpr (DERIV) {
            // this thread's tile row: its weight and its gradient's atom
            int64_t pos = -1;
            if (multi) {
                if (cs + tid < n_at)
                    pos = sbase[0] + cs + tid;
            } else if (xr) {
                int lo = 0, hi = n_seg - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sstart[mid] <= tid)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                pos = sbase[lo] + (tid - sstart[lo]);
            }
            if (pos >= 0 && !kdm_valid(a, pos))
                pos = -1;  // reported above; the row reads as zero
            rowf[tid] = pos >= 0 ? a.zeta * a.sw2 * a.pos_weight[pos] : 0.0;
            rowatom[tid] = pos >= 0 ? a.grad_atom[a.pos_grad[pos]] : -1;
        }
        __syncthreads();
        knm_gemm<BN>(acc, lds, xr, a.XM, col0, a.M, a.d);

        if constexpr (DERIV) {
            // d k / dr = zeta sigma_w^2 (x_i . x_j)^(zeta - 1) (x' . x_j), times the
            // position's weight: applied below as the values are parked
        } else {
            // k = sigma_w^2 g^zeta, in registers.
#pragma unroll
            for (int i = 0; i < KS::FM; ++i)
#pragma unroll
                for (int j = 0; j < KS::FN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[i][j][e] = a.sw2 * ipow(acc[i][j][e], a.zeta);
        }

        double *E = lds;  // [256][EPLD], reused after the GEMM
        for (int p = 0; p < (KNM_BN + EPC - 1) / EPC; ++p) {
            // waves owning columns [p*16, p*16+16) park their values in LDS
            if (wn == (p * EPC) / KS::TN) {
#pragma unroll
                for (int i = 0; i < KS::FM; ++i)
#pragma unroll
                    for (int j = 0; j < KS::FN; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int cl = acc_col<KS>(wn, j, lane, e) - p * EPC;
                            if (cl >= 0 && cl < EPC) {
                                const int r = acc_row<KS>(wm, i, lane, e);
                                double v = acc[i][j][e];
                                if constexpr (DERIV) {
                                    // (rowf / rowatom were written before the GEMM's barriers)
                                    const int64_t at = rowatom[r], colg = col0 + p * EPC + cl;
                                    const double dv = (a.D && at >= 0 && colg < a.M) ? a.D[at * a.ldd + colg] : 1.0;
                                    v = v * (rowf[r] * dv);
                                }
                                E[r * EPLD + cl] = v;
                            }
                        }
            }
            __syncthreads();
            if (!multi) {
                for (int item = tid; item < n_seg * EPC; item += KS::NT) {
                    const int s = item % n_seg, c = item / n_seg;
                    const int64_t colg = col0 + p * EPC + c;
                    if (colg >= a.M)
                        continue;
                    // in atom order; the loads of 8 (then 4) rows are issued together
                    const double sg = sig(s);
                    const int a1 = sstart[s + 1];
                    int r = sstart[s];
                    double sum = 0.0;
                    for (; r + 8 <= a1; r += 8) {
                        double v[8];
#pragma unroll
                        for (int k = 0; k < 8; ++k)
                            v[k] = E[(r + k) * EPLD + c];
#pragma unroll
                        for (int k = 0; k < 8; ++k)
                            sum += v[k];
                    }
                    if (r + 4 <= a1) {
                        double v[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            v[k] = E[(r + k) * EPLD + c];
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            sum += v[k];
                        r += 4;
                    }
                    for (; r < a1; ++r)
                        sum += E[r * EPLD + c];
                    emit(s, colg, sum, sg);
                }
            } else if (tid < EPC) {
                const int c = tid;
                const int64_t colg = col0 + p * EPC + c;
                const int nr = (int)((n_at - cs) < KNM_BM ? (n_at - cs) : KNM_BM);
                double sum = 0.0;
                for (int r = 0; r < nr; ++r)
                    sum += E[r * EPLD + c];
                const double tot = first ? sum : carry[p * EPC + c] + sum;
                carry[p * EPC + c] = tot;
                if (last && colg < a.M)
                    emit(0, colg, tot, sig(0));
            }
            __syncthreads();
        }
    }
}

template <int BN>
__global__ __launch_bounds__(256, 2) void knm_kernel(KnmArgs a) { knm_body<BN>(a, blockIdx.x); }

// Derivative observation rows: the K_NM tile loop over the observations' positions.
__global__ __launch_bounds__(256, 2) void kdm_kernel(KnmArgs a) { knm_body<64, true>(a, blockIdx.x); }

// The K_NM of several fits in one grid: fit i owns workgroups [base[i], base[i+1]).
template <int BN>
__global__ __launch_bounds__(256, 2) void knm_group_kernel(KnmGroup g)
{
    const int64_t b = blockIdx.x;
    int i = 0;
    while (i + 1 < g.n && b >= g.base[i + 1])
        ++i;
    knm_body<BN>(g.f[i], b - g.base[i]);
}

// ---------------------------------------------------------------------------
// Prediction (Eqs. 1-2): y_A = sum_{i in A} sum_j c_j sigma_w^2 (x_i . x_j)^zeta.
// Workgroup w owns configurations [w*C, (w+1)*C); it walks their atoms in
// chunks of 256, accumulates each atom's energy over all sparse tiles in LDS
// (the atom-by-sparse covariances stay in registers), then one thread per
// configuration adds its atoms' energies in atom order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 2) void predict_kernel(const double *__restrict__ X, const int64_t *offsets,
                                                      int64_t N, int64_t n_atoms, const double *__restrict__ XM,
                                                      int64_t M, int d, int zeta, double sw2,
                                                      const double *__restrict__ c, double *y, int64_t C,
                                                      int32_t *status)
{
    __shared__ double lds[2 * KS::STAGE];
    __shared__ double eps[KNM_BM];
    __shared__ double part[KS::WN][KNM_BM];
    __shared__ int bad_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / KS::WN, wn = wave % KS::WN;
    const int64_t cfg_lo = (int64_t)blockIdx.x * C;
    int64_t cfg_hi = cfg_lo + C;
    if (cfg_hi > N)
        cfg_hi = N;
    if (cfg_lo >= cfg_hi)
        return;
    const int ncfg = (int)(cfg_hi - cfg_lo);
    // Validate this workgroup's offsets before any descriptor is read: each of its
    // configurations must be a range inside [0, n_atoms) (so every row read is in
    // bounds); offsets[0] = 0 and offsets[N] = n_atoms are checked by the first
    // and last workgroup.  A violation gives NaN energies for the workgroup's
    // configurations and GAP_EINVAL in the status word (when there is one).
    if (tid == 0)
        bad_s = 0;
    __syncthreads();
    int64_t my_lo = 0, my_hi = 0;
    if (tid < ncfg) {
        my_lo = offsets[cfg_lo + tid];
        my_hi = offsets[cfg_lo + tid + 1];
        if (my_lo < 0 || my_hi < my_lo || my_hi > n_atoms)
            bad_s = 1;
    }
    if (tid == 0 && ((cfg_lo == 0 && offsets[0] != 0) || (cfg_hi == N && offsets[N] != n_atoms)))
        bad_s = 1;
    __syncthreads();
    if (bad_s) {
        if (tid < ncfg)
            y[cfg_lo + tid] = __builtin_nan("");
        if (tid == 0 && status)
            set_status(status, DST_EINVAL);
        return;
    }
    const int64_t atom_lo = offsets[cfg_lo], atom_hi = offsets[cfg_hi];
    double ysum = 0.0;
    const int64_t n_ct = (M + KNM_BN - 1) / KNM_BN;
    d4 acc[KS::FM][KS::FN];
    for (int64_t cs = atom_lo; cs < atom_hi; cs += KNM_BM) {
        __syncthreads();  // the previous chunk's sums have read eps
        if (tid < KNM_BM)
            eps[tid] = 0.0;
        for (int64_t ct = 0; ct < n_ct; ++ct) {
            const int64_t col0 = ct * KNM_BN;
            __syncthreads();
            knm_gemm<KNM_BN>(acc, lds, (cs + tid < atom_hi) ? X + (cs + tid) * (int64_t)d : nullptr, XM, col0, M,
                             d);
            double cw[KS::FN][4];
#pragma unroll
            for (int j = 0; j < KS::FN; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t col = col0 + acc_col<KS>(wn, j, lane, e);
                    cw[j][e] = (col < M) ? c[col] : 0.0;
                }
#pragma unroll
            for (int i = 0; i < KS::FM; ++i) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < KS::FN; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        s += cw[j][e] * (sw2 * ipow(acc[i][j][e], zeta));
                // the 4 lanes that differ in l % 4 share this row
                s += __shfl_xor(s, 1, 64);
                s += __shfl_xor(s, 2, 64);
                if ((lane & 3) == 0)
                    part[wn][acc_row<KS>(wm, i, lane, 0)] = s;
            }
            __syncthreads();
            if (tid < KNM_BM) {
                double add = 0.0;
#pragma unroll
                for (int q = 0; q < KS::WN; ++q)
                    add += part[q][tid];
                eps[tid] += add;
            }
        }
        __syncthreads();
        if (tid < ncfg) {
            const int64_t lo = my_lo > cs ? my_lo : cs;
            const int64_t hi = my_hi < cs + KNM_BM ? my_hi : cs + KNM_BM;
            for (int64_t a = lo; a < hi; ++a)
                ysum += eps[a - cs];
        }
    }
    if (tid < ncfg)
        y[cfg_lo + tid] = ysum;
}

hipError_t launch_predict(const double *X, int64_t n_atoms, const int64_t *offsets, int64_t N,
                          const double *XM, int64_t M, int d, int zeta, double sw2, const double *c,
                          double *y, int32_t *status, hipStream_t s)
{
    if (N <= 0)
        return hipSuccess;
    int64_t C = n_atoms > 0 ? (224 * N) / n_atoms : N;
    if (C < 1)
        C = 1;
    if (C > 256)
        C = 256;
    const int64_t grid = (N + C - 1) / C;
    hipLaunchKernelGGL(predict_kernel, dim3((unsigned)grid), dim3(KS::NT), 0, s, X, offsets, N, n_atoms, XM, M,
                       d, zeta, sw2, c, y, C, status);
    return hipGetLastError();
}

hipError_t launch_plan_tiles(const int64_t *offsets, int64_t N, int64_t n_atoms, const KnmPlan &p, int64_t max_tiles,
                             int32_t *status, hipStream_t s)
{
    const int64_t nc = knm_plan_chunks(N);
    hipLaunchKernelGGL(plan_chunk_kernel, dim3((unsigned)nc), dim3(256), 0, s, offsets, N, n_atoms, p.cfg_list,
                       p.lstart, p.lcount, status);
    hipLaunchKernelGGL(plan_publish_kernel, dim3((unsigned)nc), dim3(256), 0, s, (const int32_t *)p.lstart,
                       (const int32_t *)p.lcount, nc, N, p.tile_start, p.n_tiles, max_tiles, status);
    return hipGetLastError();
}

static int bn_of(const KnmArgs &a) { return a.bn == 32 ? 32 : 64; }

hipError_t launch_knm_group(const KnmArgs *fits, const int64_t *max_tiles, int n, hipStream_t s)
{
    for (int bn : {64, 32}) {  // one grid per column-tile width
        KnmGroup g{};
        auto flush = [&]() {
            if (g.n > 0 && g.base[g.n] > 0) {
                if (bn == 64)
                    hipLaunchKernelGGL(knm_group_kernel<64>, dim3((unsigned)g.base[g.n]), dim3(256), 0, s, g);
                else
                    hipLaunchKernelGGL(knm_group_kernel<32>, dim3((unsigned)g.base[g.n]), dim3(256), 0, s, g);
            }
            g = KnmGroup{};
        };
        for (int i = 0; i < n; ++i) {
            if (bn_of(fits[i]) != bn)
                continue;
            KnmArgs a = fits[i];
            a.n_ct = (a.M + bn - 1) / bn;
            const int64_t total = max_tiles[i] * a.n_ct;
            a.total_pad = (total + 7) & ~int64_t(7);
            g.f[g.n] = a;
            g.base[g.n + 1] = g.base[g.n] + a.total_pad;
            if (++g.n == KNM_GROUP)
                flush();
        }
        flush();
    }
    return hipGetLastError();
}

hipError_t launch_kdm(KnmArgs a, int64_t max_tiles, hipStream_t s)
{
    a.n_ct = (a.M + 63) / 64;
    a.total_pad = (max_tiles + 7) / 8 * 8 * a.n_ct;  // whole rounds of 8 tiles (see knm_body)
    if (a.total_pad == 0)
        return hipSuccess;
    hipLaunchKernelGGL(kdm_kernel, dim3((unsigned)a.total_pad), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_knm(KnmArgs a, int64_t max_tiles, hipStream_t s)
{
    const int bn = bn_of(a);
    a.n_ct = (a.M + bn - 1) / bn;
    const int64_t total = max_tiles * a.n_ct;
    a.total_pad = (total + 7) & ~int64_t(7);
    if (a.total_pad == 0)
        return hipSuccess;
    if (bn == 64)
        hipLaunchKernelGGL(knm_kernel<64>, dim3((unsigned)a.total_pad), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(knm_kernel<32>, dim3((unsigned)a.total_pad), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace gap
