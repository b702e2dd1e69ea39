// FP64-accurate K_NM on INT8 MFMA (Ozaki scheme).  The descriptor dot
// products of the K_MN definition (Sec. Theory) are formed exactly in integer
// arithmetic from 8-bit slices of the FP64 values, then the power, the
// per-configuration segment sum and the Sigma^-1/2 row scale run in FP64 as in
// the FP64 build.
//
// Slicing (Ozaki, Ogita, Oishi & Rump 2012, with integer slice products as in
// Ootomo, Ozaki & Yokota 2024).  Row r of a descriptor array gets an exponent
// e_r with max_k |x_rk| < 2^e_r, and every entry becomes the integer
// N = rint(x 2^(54 - e_r)), |N| < 2^54, so x = N 2^(e_r - 54) up to half a unit
// of 2^(e_r - 54).  N is written in OZ_S = 7 balanced base-256 digits,
// N = sum_t D_t 256^(6 - t) with D_t in [-128, 127] (t = 0 the most significant,
// |D_0| <= 64).  Then
//   x_i . x_j = 2^(e_i + e_j - 12) sum_delta 2^(-8 delta) S_delta,
//   S_delta = sum_{t + u = delta} D_t(x_i) . D_u(x_j),
// with every S_delta exact in INT32 (at most 7 products of dp <= 4096 terms of
// at most 2^14 each).  Diagonals delta <= 6 are kept (28 slice products): the
// first dropped one is below 2^-56 of the leading term, so the dot product
// carries the error of the rounding to 54 bits, about FP64's own.
#include "knm.h"

namespace gap {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

constexpr int OZ_S = 7;      // slices
constexpr int OZ_BITS = 54;  // |N| < 2^54
constexpr int OZ_KC = 32;    // bytes of k per chunk of the slice layout (one MFMA's k)

int knm_oz_dpad(int d) { return (d + OZ_KC - 1) / OZ_KC * OZ_KC; }
int knm_oz_slices() { return OZ_S; }

// One wave per row: the row's exponent, then its digits, four entries (one
// 32-bit word per slice) per lane and step.  Layout, chunk-major so that the
// 32-byte k-chunks of consecutive rows are contiguous: byte k of slice t of
// row r is at out + t * rows * dp + (k / 32) * rows * 32 + r * 32 + k % 32.
// Entries k >= d are zero.
__global__ __launch_bounds__(256) void oz_split_kernel(const double *__restrict__ x, int64_t rows, int d, int dp,
                                                       int8_t *__restrict__ out, int32_t *__restrict__ ex)
{
    const int lane = threadIdx.x & 63;
    const int64_t slice = rows * (int64_t)dp;
    const int64_t waves = (int64_t)gridDim.x * 4;
    for (int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6; r < rows; r += waves) {
        const double *src = x + r * (int64_t)d;
        double m = 0.0;
        for (int k = lane; k < d; k += 64)
            m = fmax(m, fabs(src[k]));
        for (int o = 32; o > 0; o >>= 1)
            m = fmax(m, __shfl_xor(m, o));
        int e = 0;
        if (m > 0.0)
            (void)frexp(m, &e);  // m = f 2^e, f in [0.5, 1): every |x| < 2^e
        if (lane == 0)
            ex[r] = e;
        for (int w = lane; w < dp / 4; w += 64) {
            uint32_t word[OZ_S];
#pragma unroll
            for (int t = 0; t < OZ_S; ++t)
                word[t] = 0u;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 4 * w + q;
                int64_t n = k < d ? (int64_t)rint(ldexp(src[k], OZ_BITS - e)) : 0;
#pragma unroll
                for (int t = OZ_S - 1; t > 0; --t) {
                    const int8_t dg = (int8_t)(uint8_t)(n & 0xff);  // n - dg is a multiple of 256
                    word[t] |= (uint32_t)(uint8_t)dg << (8 * q);
                    n = (n - dg) >> 8;
                }
                word[0] |= (uint32_t)(uint8_t)(int8_t)n << (8 * q);
            }
            const int64_t pos = (int64_t)(w / 8) * rows * OZ_KC + r * OZ_KC + 4 * (w % 8);
#pragma unroll
            for (int t = 0; t < OZ_S; ++t)
                *reinterpret_cast<uint32_t *>(out + t * slice + pos) = word[t];
        }
    }
}

// ---------------------------------------------------------------------------
// Tile: 128 atoms (a chunk of the plan's tile of up to 256 atoms, whole
// configurations) x 64 sparse points, 512 threads = 8 waves of 32 x 32 (4 along
// the atoms, 2 along the sparse points), two waves per SIMD.  Each wave holds the
// seven diagonals' exact INT32 sums of its 32 x 32 outputs at once (seven
// accumulator blocks, 112 registers), so the k loop streams every operand byte
// once: a stage holds one 32-byte k-chunk of all seven slices of both operands
// (42 KB), and its 28 slice products run from LDS while the next stage's direct
// global-to-LDS loads are in flight (two stages).  Per k-chunk a wave reads its
// seven B fragments once and keeps them, and one A fragment per slice t.  The
// diagonals are folded into FP64 (exact scaling by 2^(-8 delta)) once, after the
// k loop.  A workgroup takes OCT consecutive column tiles of one atom tile, and
// for each column tile the atom tile's chunks of 128 rows in order; a
// configuration that runs across a chunk boundary carries its partial sums in
// LDS.
//
// Operand layout of v_mfma_i32_32x32x32_i8: lane l supplies row (A) or column
// (B) l % 32 and the sixteen k of half l / 32; accumulator element e of lane l
// is C(8 (e / 4) + 4 (l / 32) + e % 4, l % 32).
// ---------------------------------------------------------------------------
constexpr int OBM = 128;                 // atoms per chunk
constexpr int OBN = 64;                  // sparse points per tile
constexpr int ONT = 512;
constexpr int OCT = 8;                   // column tiles per workgroup
constexpr int OSA = OBM * OZ_KC;         // one slice's A rows in a stage: 4 KB
constexpr int OSB = OBN * OZ_KC;         // one slice's B rows: 2 KB
constexpr int OSTAGE = OZ_S * (OSA + OSB);  // A slices 0..6, then B slices 0..6: 42 KB
constexpr int OITEMS = OSTAGE / 1024;    // 1 KB loads per stage: 28 of A, then 14 of B
constexpr int OEPLD = OBN + 1;           // the epilogue's row stride (all 64 columns at once)
static_assert(ONT == 512 && OSA == 4 * 1024 && OSB == 2 * 1024, "load mapping: A parts = wave % 4, B = wave % 2");
static_assert(2 * OBM == KNM_BM, "a plan tile is two chunks (or one configuration in several)");

struct KnmOzArgs {
    const int8_t *X, *XM;     // slices (chunk-major, see oz_split_kernel)
    int64_t x_slice, xm_slice;
    int64_t x_chunk, xm_chunk;  // rows * 32: bytes between consecutive k-chunks of a slice
    const int32_t *xe, *xme;  // row exponents
    int nk;                   // k-chunks per row
    const int64_t *offsets;
    const int32_t *tile_start, *cfg_list, *n_tiles_dev;
    int64_t M;
    int zeta;
    double sw2;
    const double *sigma;
    double *out;              // column-major: out[col * ldo + configuration]
    int64_t ldo;
    int64_t n_ct, n_cg;
};

// Half of a stage row that holds k-half h of row r: the halves of rows are
// swapped in a pattern that gives the 16 rows read by one group of lanes
// distinct banks.
DEV int oz_half(int r, int h) { return h ^ (((r >> 2) ^ (r >> 3)) & 1); }

DEV double ipow_oz(double g, int zeta)
{
    double p = g;
    for (int z = 1; z < zeta; ++z)
        p *= g;
    return p;
}

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(3))) char lds_char;

__global__ __launch_bounds__(ONT) __attribute__((amdgpu_waves_per_eu(2, 2))) void knm_oz_kernel(KnmOzArgs a)
{
    // two stages as separate arrays: loads into one never alias the reads of the other
    __shared__ __align__(16) unsigned char stage0[OSTAGE], stage1[OSTAGE];
    __shared__ double E[OBM * OEPLD];
    __shared__ double carry[2][OBN];  // partial sums of the configuration crossing a chunk boundary
    __shared__ int32_t sstart[KNM_MAX_SEG + 1];
    __shared__ int64_t sbase[KNM_MAX_SEG];
    __shared__ int32_t srow[KNM_MAX_SEG];
    __shared__ int32_t scan[KNM_MAX_SEG];
    __shared__ int32_t sexp[2][OBM];  // row and column exponents, by unit parity
    __shared__ int32_t cexp[2][OBN];

    const int64_t n_tiles = (int64_t)*a.n_tiles_dev;
    const int64_t total = n_tiles * a.n_cg;
    const int64_t total_pad = (total + 7) & ~int64_t(7);
    if ((int64_t)blockIdx.x >= total_pad)
        return;
    const int64_t lw = xcd_remap(blockIdx.x, total_pad);
    if (lw >= total)
        return;
    const int64_t t_id = lw / a.n_cg, cg = lw % a.n_cg;
    const int64_t ct_lo = cg * OCT, ct_hi = (ct_lo + OCT) < a.n_ct ? (ct_lo + OCT) : a.n_ct;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // segments (configurations) of the tile and their atom offsets within it
    const int64_t p0 = a.tile_start[t_id];
    const int n_seg = (int)(a.tile_start[t_id + 1] - p0);
    if (tid < KNM_MAX_SEG) {
        int64_t sz = 0;
        if (tid < n_seg) {
            const int32_t cfg = a.cfg_list[p0 + tid];
            const int64_t lo = a.offsets[cfg];
            sz = a.offsets[cfg + 1] - lo;
            sbase[tid] = lo;
            srow[tid] = cfg;
        }
        scan[tid] = (int32_t)sz;
    }
    __syncthreads();
    for (int off = 1; off < KNM_MAX_SEG; off <<= 1) {
        int32_t v = 0;
        if (tid < KNM_MAX_SEG && tid >= off)
            v = scan[tid - off];
        __syncthreads();
        if (tid < KNM_MAX_SEG)
            scan[tid] += v;
        __syncthreads();
    }
    if (tid < KNM_MAX_SEG)
        sstart[tid + 1] = scan[tid];
    if (tid == 0)
        sstart[0] = 0;
    __syncthreads();
    const int64_t n_at = sstart[n_seg];

    auto emit = [&](int s, int64_t colg, double sum) {
        const int64_t row = srow[s];
        a.out[colg * a.ldo + row] = sum / a.sigma[row];
    };
    if (n_at == 0) {  // only empty configurations: their sums are zero
        const int ncol = (int)((ct_hi - ct_lo) * OBN);
        for (int item = tid; item < n_seg * ncol; item += ONT) {
            const int s = item % n_seg, c = item / n_seg;
            const int64_t colg = ct_lo * OBN + c;
            if (colg < a.M)
                emit(s, colg, 0.0);
        }
        return;
    }
    const bool multi = n_at > KNM_BM;  // then n_seg == 1: one configuration in several chunks

    // the segment holding tile row r (r < n_at)
    auto seg_of = [&](int64_t r) -> int {
        int lo = 0, hi = n_seg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sstart[mid] <= r)
                lo = mid;
            else
                hi = mid - 1;
        }
        return lo;
    };
    auto atom_of = [&](int64_t r) -> int64_t {  // descriptor row of tile row r, -1 past the tile
        if (r >= n_at)
            return -1;
        if (multi)
            return sbase[0] + r;
        const int s = seg_of(r);
        return sbase[s] + (r - sstart[s]);
    };

    // Direct global-to-LDS loads of 1 KB each (lane l lands at 16 l): load i of a
    // stage is A slice i / 4, rows 32 (i % 4) ..  (i < 28), else B slice (i - 28) / 2,
    // rows 32 ((i - 28) % 2) ..; wave w issues loads w, w + 8, .., so it always
    // loads the A rows 32 (w % 4) + l / 2 and the B rows 32 (w % 2) + l / 2, lane l
    // the k-half that lands in stage half l % 2 (oz_half).
    const int arow = 32 * (wave & 3) + (lane >> 1), brow = 32 * (wave & 1) + (lane >> 1);
    const int ahalf = oz_half(arow, lane & 1), bhalf = oz_half(brow, lane & 1);
    // fragment reads: A rows 32 wm + l % 32, B columns 32 wn + l % 32
    const int fr = 32 * wm + (lane & 31), fc = 32 * wn + (lane & 31);
    const int a_off = fr * OZ_KC + 16 * oz_half(fr, lane >> 5);
    const int b_off = OZ_S * OSA + fc * OZ_KC + 16 * oz_half(fc, lane >> 5);
    const int nk = a.nk;

    // Units: (column tile, chunk of 128 tile rows), chunks inner.  A unit's setup (its
    // load offsets and exponents, double-buffered by unit parity) and its first stage's
    // loads are issued before the previous unit's epilogue, which then hides them.
    const int64_t n_chunks = (n_at + OBM - 1) / OBM;
    const int64_t n_units = (ct_hi - ct_lo) * n_chunks;
    int64_t aoff = 0, boff = 0;  // this lane's load offsets for the unit being loaded
    auto setup = [&](int64_t u) {
        const int64_t ct = ct_lo + u / n_chunks, cs = (u % n_chunks) * OBM;
        const int64_t col0 = ct * OBN, colb = col0 + brow;
        boff = (colb < a.M ? colb * OZ_KC : 0) + 16 * bhalf;  // past M: any valid row
        const int64_t at = atom_of(cs + arow);
        aoff = (at >= 0 ? at * OZ_KC : 0) + 16 * ahalf;  // rows past the tile: unused
        int32_t *se = sexp[u & 1], *ce = cexp[u & 1];
        if (tid < OBM) {
            const int64_t ar = atom_of(cs + tid);
            se[tid] = ar >= 0 ? a.xe[ar] : 0;
        } else if (tid < OBM + OBN) {
            const int c = tid - OBM;
            ce[c] = (col0 + c < a.M) ? a.xme[col0 + c] : 0;
        }
    };
    auto issue = [&](int kc, unsigned char *stg) {  // k-chunk kc of all fourteen slice tiles
        const int8_t *xa = a.X + kc * a.x_chunk + aoff;
        const int8_t *xb = a.XM + kc * a.xm_chunk + boff;
#pragma unroll
        for (int m = 0; m < (OITEMS + 7) / 8; ++m) {
            const int i = wave + 8 * m;
            if (i < 4 * OZ_S) {
                const int t = i >> 2;
                __builtin_amdgcn_global_load_lds((const void *)(xa + t * a.x_slice),
                                                 (lds_void *)(stg + t * OSA + 1024 * (i & 3)), 16, 0, 0);
            } else if (i < OITEMS) {
                const int j = i - 4 * OZ_S, u = j >> 1;
                __builtin_amdgcn_global_load_lds((const void *)(xb + u * a.xm_slice),
                                                 (lds_void *)(stg + OZ_S * OSA + u * OSB + 1024 * (j & 1)), 16, 0,
                                                 0);
            }
        }
    };

    i32x16 acc[OZ_S];
    setup(0);
    issue(0, stage0);
    for (int64_t unit = 0; unit < n_units; ++unit) {
        const int64_t ct = ct_lo + unit / n_chunks, cs = (unit % n_chunks) * OBM;
        const int64_t col0 = ct * OBN;
        const int32_t *se = sexp[unit & 1], *ce_exp = cexp[unit & 1];
        {
#pragma unroll
            for (int dl = 0; dl < OZ_S; ++dl)
                acc[dl] = i32x16{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};

            auto compute = [&](const unsigned char *stg) {  // the 28 slice products of one k-chunk
                i32x4 bf[OZ_S];
#pragma unroll
                for (int u = 0; u < OZ_S; ++u)
                    bf[u] = *reinterpret_cast<const i32x4 *>(stg + u * OSB + b_off);
#pragma unroll
                for (int t = 0; t < OZ_S; ++t) {
                    const i32x4 af = *reinterpret_cast<const i32x4 *>(stg + t * OSA + a_off);
#pragma unroll
                    for (int u = 0; u + t < OZ_S; ++u)
                        acc[t + u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af, bf[u], acc[t + u], 0, 0, 0);
                }
                // schedule: four reads ahead, then one read per MFMA until the reads are issued
                __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
                for (int r = 0; r < 2 * OZ_S - 4; ++r) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x008, OZ_S * (OZ_S + 1) / 2 - (2 * OZ_S - 4), 0);
            };

            for (int kc = 0; kc < nk; kc += 2) {
                __syncthreads();  // (waits for this wave's loads) stage 0 holds chunk kc; stage 1 is free
                if (kc + 1 < nk)
                    issue(kc + 1, stage1);
                compute(stage0);
                if (kc + 1 < nk) {
                    __syncthreads();  // stage 1 holds chunk kc + 1; stage 0 is free
                    if (kc + 2 < nk)
                        issue(kc + 2, stage0);
                    compute(stage1);
                }
            }

            __syncthreads();  // every wave is done with the stages
            if (unit + 1 < n_units) {  // the next unit's setup and first stage, hidden by this epilogue
                setup(unit + 1);
                issue(0, stage0);
            }
            // This chunk, rows [cs, ce), handles the segments that meet it, the empty ones
            // at positions in [cs, ce) and, if it is the last, the empty ones at n_at:
            // segments [s_lo, s_hi) with s_lo the first that ends after cs or starts at
            // or after it, s_hi the first that starts at or after ce.
            const int64_t ce = (cs + OBM < n_at) ? cs + OBM : n_at;
            auto first_seg = [&](auto pred) {  // first s in [0, n_seg) with pred(s), else n_seg
                int lo = 0, hi = n_seg;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (pred(mid))
                        hi = mid;
                    else
                        lo = mid + 1;
                }
                return lo;
            };
            const int s_lo = first_seg([&](int q) { return sstart[q] >= cs || sstart[q + 1] > cs; });
            const int s_hi = (ce == n_at) ? n_seg : first_seg([&](int q) { return sstart[q] >= ce; });
            const int n_cs = s_hi - s_lo;
            const double *cin = carry[unit & 1];  // written by the previous unit
            double *cout = carry[(unit + 1) & 1];
            // Epilogue: the diagonals folded into FP64, g = 2^(e_i + e_j - 12) sum,
            // k = sigma_w^2 g^zeta into E (every wave its block), then the sums over each
            // configuration's atoms in atom order (the next chunk's first barrier ends it).
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                double sum = 0.0;
#pragma unroll
                for (int dl = OZ_S - 1; dl >= 0; --dl)
                    sum = fma((double)acc[dl][e], ldexp(1.0, -8 * dl), sum);
                const int r = 32 * wm + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                const int c = 32 * wn + (lane & 31);
                const double g = ldexp(sum, se[r] + ce_exp[c] - 12);
                E[r * OEPLD + c] = a.sw2 * ipow_oz(g, a.zeta);
            }
            __syncthreads();
            for (int item = tid; item < n_cs * OBN; item += ONT) {
                const int s = s_lo + item / OBN, c = item % OBN;
                const int64_t lo = sstart[s] > cs ? sstart[s] : cs;
                const int64_t hi = sstart[s + 1] < ce ? sstart[s + 1] : ce;
                double part = (sstart[s] < cs) ? cin[c] : 0.0;  // began in an earlier chunk
                for (int64_t r = lo; r < hi; ++r)  // atom order
                    part += E[(r - cs) * OEPLD + c];
                const int64_t colg = col0 + c;
                if (sstart[s + 1] > ce)  // continues in the next chunk
                    cout[c] = part;
                else if (colg < a.M)
                    emit(s, colg, part);
            }
        }
    }  // units
}

hipError_t launch_oz_split(const double *x, int64_t rows, int d, int8_t *out, int32_t *ex, hipStream_t s)
{
    if (rows <= 0)
        return hipSuccess;
    int64_t g = (rows + 3) / 4;
    if (g > 65536)
        g = 65536;
    hipLaunchKernelGGL(oz_split_kernel, dim3((unsigned)g), dim3(256), 0, s, x, rows, d, knm_oz_dpad(d), out, ex);
    return hipGetLastError();
}

hipError_t launch_knm_oz(const KnmOzLaunch &l, hipStream_t s)
{
    KnmOzArgs a{};
    const int dp = knm_oz_dpad(l.d);
    a.nk = dp / OZ_KC;
    a.X = l.X;
    a.XM = l.XM;
    a.x_slice = l.n_atoms * (int64_t)dp;
    a.xm_slice = l.M * (int64_t)dp;
    a.x_chunk = l.n_atoms * (int64_t)OZ_KC;
    a.xm_chunk = l.M * (int64_t)OZ_KC;
    a.xe = l.xe;
    a.xme = l.xme;
    a.offsets = l.offsets;
    a.tile_start = l.tile_start;
    a.cfg_list = l.cfg_list;
    a.n_tiles_dev = l.n_tiles_dev;
    a.M = l.M;
    a.zeta = l.zeta;
    a.sw2 = l.sw2;
    a.sigma = l.sigma;
    a.out = l.out;
    a.ldo = l.ldo;
    a.n_ct = (l.M + OBN - 1) / OBN;
    a.n_cg = (a.n_ct + OCT - 1) / OCT;
    const int64_t total = l.max_tiles * a.n_cg;
    const int64_t total_pad = (total + 7) & ~int64_t(7);
    if (total_pad == 0 || a.nk == 0)
        return hipSuccess;
    hipLaunchKernelGGL(knm_oz_kernel, dim3((unsigned)total_pad), dim3(ONT), 0, s, a);
    return hipGetLastError();
}

}  // namespace gap
