// Shared device helpers of the GAP fit library (gfx950 / CDNA4 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DEV __device__ __forceinline__

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Device status word values (same numbering as gap_status).
enum : int32_t {
    DST_OK = 0,
    DST_EINVAL = 1,
    DST_ENOTPD = 3,
    DST_ENONFINITE = 4,
    DST_ENOCONV = 5,
    DST_EDEVICE = 6,  // a device-side wait was abandoned
    DST_ERANK = 8,    // a QR panel's Gram matrix lost positive definiteness
};

// Record the first failure seen on the device; later ones do not overwrite it.
DEV void set_status(int32_t *status, int32_t code)
{
    atomicCAS(reinterpret_cast<int *>(status), 0, code);
}

// ---------------------------------------------------------------------------
// "Last workgroup" completion pattern: every workgroup publishes its partial
// results, then one arrival counter tells the last one that all partials are
// visible.  The counter is reset by that last workgroup, ready for the next
// launch that uses it.  Returns true in every thread of the last workgroup.
// ---------------------------------------------------------------------------
DEV bool arrive_last(unsigned *counter, unsigned nblocks, int *flag_lds)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        int last = (prev == nblocks - 1);
        if (last)
            __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *flag_lds = last;
    }
    __syncthreads();
    int last = *flag_lds;
    if (last)
        __atomic_thread_fence(__ATOMIC_ACQUIRE);  // see the other workgroups' partials
    return last != 0;
}

// Publish this workgroup's global writes before it arrives (all threads call).
DEV void release_writes() { __atomic_thread_fence(__ATOMIC_RELEASE); }

// Wave-wide sum with a fixed butterfly order (deterministic).
DEV double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// FP64 MFMA tile machinery.
//
// A workgroup computes a BM x BN tile C = sum_k Aop(m, k) * Bop(n, k).  Both
// operands are staged in LDS "K-major": As[k * LDA + m], Bs[k * LDB + n].  The
// WM x WN waves each own a TM x TN sub-tile made of FM x FN blocks of 16x16.
//
// By default each 16x16x4 block product is done with four
// v_mfma_f64_4x4x4_4b_f64 (the K_NM's loop measured 3 % faster with them).
// That instruction holds four independent 4x4x4 products in the lane groups
// g = (l/4)%4: A(m, k) of block g at lane 16k + 4g + (m%4), B(k, n) at lane
// 16k + 4g + (n%4), result (m, n) at lane 16(m%4) + 4g + (n%4).  With the A
// register holding A(l%16, l/16) (rows 4g..4g+3 in group g) and the s-th B
// register holding B(l/16, 4s + l%4) in every group, instruction s computes
// the 4x4 blocks (row group g, column group s) for g = 0..3; the four
// instructions together cover the 16x16 block.  The four lanes of a k-row
// that share l%4 read the same B element (an LDS broadcast), so a B read moves
// 16 distinct values.  Accumulator element s of lane l is
// C(4g + l/16, 4s + l%4) with g = (l/4)%4 (layout measured on gfx950).
//
// Shapes with M16 set use one v_mfma_f64_16x16x4_f64 per 16x16 block and 4 k
// instead: lane l supplies A(l%16, l/16) and B(l/16, l%16), and accumulator
// element e of lane l is C(l/16 + 4e, l%16) (measured on gfx950; the FP32
// instruction's rows run the other way).  A wave's 64 x 64 tile then takes
// 4 + 4 LDS reads per 16 instructions instead of 4 + 16 per 64.
// ---------------------------------------------------------------------------
template <int BM_, int BN_, int BK_, int WM_, int WN_, bool M16_ = false>
struct TileShape {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
    static constexpr bool M16 = M16_;
    static constexpr int NT = WM * WN * 64;
    static constexpr int TM = BM / WM, TN = BN / WN;
    static constexpr int FM = TM / 16, FN = TN / 16;
    static constexpr int PAD = 16;  // row offset of 32 banks between the k-rows read by one MFMA
    static constexpr int LDA = BM + PAD, LDB = BN + PAD;
    static constexpr int A_ELEMS = BK * LDA, B_ELEMS = BK * LDB;
    static constexpr int STAGE = A_ELEMS + B_ELEMS;
    static_assert(TM % 16 == 0 && TN % 16 == 0, "wave tile must be whole 16x16 blocks");
    static_assert(BK % 4 == 0, "BK must be a multiple of the MFMA K (4)");
};

template <class S>
DEV void zero_acc(d4 (&acc)[S::FM][S::FN])
{
#pragma unroll
    for (int i = 0; i < S::FM; ++i)
#pragma unroll
        for (int j = 0; j < S::FN; ++j)
            acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
}

// Column (within a 16-wide block) that B register s of lane l carries.
DEV int bcol16(int lane, int s) { return 4 * s + (lane & 3); }

template <class S>
DEV void mma_stage(const double *__restrict__ As, const double *__restrict__ Bs,
                   d4 (&acc)[S::FM][S::FN], int wm, int wn, int lane)
{
#pragma unroll
    for (int kk = 0; kk < S::BK; kk += 4) {
        const int kr = kk + (lane >> 4);
        double a[S::FM];
#pragma unroll
        for (int i = 0; i < S::FM; ++i)
            a[i] = As[kr * S::LDA + wm * S::TM + i * 16 + (lane & 15)];
        if constexpr (S::M16) {
            double b[S::FN];
#pragma unroll
            for (int j = 0; j < S::FN; ++j)
                b[j] = Bs[kr * S::LDB + wn * S::TN + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < S::FM; ++i)
#pragma unroll
                for (int j = 0; j < S::FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        } else {
#pragma unroll
            for (int j = 0; j < S::FN; ++j) {
                double b[4];
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    b[s] = Bs[kr * S::LDB + wn * S::TN + j * 16 + bcol16(lane, s)];
#pragma unroll
                for (int i = 0; i < S::FM; ++i)
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc[i][j][s] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[i], b[s], acc[i][j][s], 0, 0, 0);
            }
        }
    }
}

// Row / column (within the workgroup tile) of accumulator element e.
template <class S>
DEV int acc_row(int wm, int i, int lane, int e)
{
    if constexpr (S::M16)
        return wm * S::TM + i * 16 + (lane >> 4) + 4 * e;
    return wm * S::TM + i * 16 + 4 * ((lane >> 2) & 3) + (lane >> 4);
}
template <class S>
DEV int acc_col(int wn, int j, int lane, int e)
{
    if constexpr (S::M16)
        return wn * S::TN + j * 16 + (lane & 15);
    return wn * S::TN + j * 16 + bcol16(lane, e);
}

// Integer power by repeated multiplication, p = g^zeta (zeta >= 1).
DEV double ipow(double g, int zeta)
{
    double p = g;
    for (int z = 1; z < zeta; ++z)
        p *= g;
    return p;
}

// Map a hardware workgroup id to a logical id so that consecutive logical ids
// run on the same XCD (workgroups are dispatched to the 8 XCDs round-robin).
// total_pad must be a multiple of 8.
DEV int64_t xcd_remap(int64_t w, int64_t total_pad)
{
    const int64_t per = total_pad >> 3;
    return (w & 7) * per + (w >> 3);
}

// ---------------------------------------------------------------------------
// Generic LDS-staged MFMA tile product over a K range [0, K):
//   acc(m, n) += sum_k fa(m, k) * fb(n, k)
// fa/fb return the operand value (0 outside the valid range).  A_KC / B_KC
// say whether consecutive k of one row are contiguous in memory (each thread
// then reads a run along k); otherwise consecutive rows are contiguous (each
// thread reads a run of rows at one k).  Double-buffered: one barrier per
// BK-slice, the next slice's global loads in flight during the MFMAs.
// ---------------------------------------------------------------------------
template <class S, bool A_KC, bool B_KC, class FA, class FB>
DEV void gemm_tile(d4 (&acc)[S::FM][S::FN], double *lds, int64_t K, FA fa, FB fb)
{
    constexpr int VA = S::BM * S::BK / S::NT;
    constexpr int VB = S::BN * S::BK / S::NT;
    static_assert(VA >= 1 && VB >= 1, "tile too small for the thread count");
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave / S::WN, wn = wave % S::WN;
    double ra[VA], rb[VB];
    auto load = [&](int64_t k0) {
        if constexpr (A_KC) {
            constexpr int TPR = S::BK / VA;
            const int row = t / TPR, kb = (t % TPR) * VA;
#pragma unroll
            for (int e = 0; e < VA; ++e)
                ra[e] = fa(row, k0 + kb + e);
        } else {
            constexpr int TPK = S::BM / VA;
            const int k = t / TPK, r0 = (t % TPK) * VA;
#pragma unroll
            for (int e = 0; e < VA; ++e)
                ra[e] = fa(r0 + e, k0 + k);
        }
        if constexpr (B_KC) {
            constexpr int TPR = S::BK / VB;
            const int row = t / TPR, kb = (t % TPR) * VB;
#pragma unroll
            for (int e = 0; e < VB; ++e)
                rb[e] = fb(row, k0 + kb + e);
        } else {
            constexpr int TPK = S::BN / VB;
            const int k = t / TPK, r0 = (t % TPK) * VB;
#pragma unroll
            for (int e = 0; e < VB; ++e)
                rb[e] = fb(r0 + e, k0 + k);
        }
    };
    auto store = [&](double *As, double *Bs) {
        if constexpr (A_KC) {
            constexpr int TPR = S::BK / VA;
            const int row = t / TPR, kb = (t % TPR) * VA;
#pragma unroll
            for (int e = 0; e < VA; ++e)
                As[(kb + e) * S::LDA + row] = ra[e];
        } else {
            constexpr int TPK = S::BM / VA;
            const int k = t / TPK, r0 = (t % TPK) * VA;
#pragma unroll
            for (int e = 0; e < VA; ++e)
                As[k * S::LDA + r0 + e] = ra[e];
        }
        if constexpr (B_KC) {
            constexpr int TPR = S::BK / VB;
            const int row = t / TPR, kb = (t % TPR) * VB;
#pragma unroll
            for (int e = 0; e < VB; ++e)
                Bs[(kb + e) * S::LDB + row] = rb[e];
        } else {
            constexpr int TPK = S::BN / VB;
            const int k = t / TPK, r0 = (t % TPK) * VB;
#pragma unroll
            for (int e = 0; e < VB; ++e)
                Bs[k * S::LDB + r0 + e] = rb[e];
        }
    };
    const int64_t nk = (K + S::BK - 1) / S::BK;
    if (nk <= 0)
        return;
    load(0);
    store(lds, lds + S::A_ELEMS);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        double *cur = lds + (kt & 1) * S::STAGE;
        double *nxt = lds + ((kt + 1) & 1) * S::STAGE;
        const bool more = kt + 1 < nk;
        if (more)
            load((kt + 1) * S::BK);
        mma_stage<S>(cur, cur + S::A_ELEMS, acc, wm, wn, lane);
        if (more)
            store(nxt, nxt + S::A_ELEMS);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Same product with run loaders: fa(r, k, v) fills v[0..VA) with a run of
// consecutive elements (along k when A_KC, else along the row index, starting
// at the given (r, k)); likewise fb with VB.  Lets the caller issue vector
// loads and keep bounds checks off the common path.
// ---------------------------------------------------------------------------
template <class S, bool A_KC, bool B_KC, class FA, class FB>
DEV void gemm_tile_runs(d4 (&acc)[S::FM][S::FN], double *lds, int64_t K, FA fa, FB fb)
{
    constexpr int VA = S::BM * S::BK / S::NT;
    constexpr int VB = S::BN * S::BK / S::NT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave / S::WN, wn = wave % S::WN;
    double ra[VA], rb[VB];
    // per-thread run origin inside the tile
    int ar, ak, br, bk;
    if constexpr (A_KC) {
        ar = t / (S::BK / VA);
        ak = (t % (S::BK / VA)) * VA;
    } else {
        ak = t / (S::BM / VA);
        ar = (t % (S::BM / VA)) * VA;
    }
    if constexpr (B_KC) {
        br = t / (S::BK / VB);
        bk = (t % (S::BK / VB)) * VB;
    } else {
        bk = t / (S::BN / VB);
        br = (t % (S::BN / VB)) * VB;
    }
    auto store = [&](double *As, double *Bs) {
#pragma unroll
        for (int e = 0; e < VA; ++e) {
            if constexpr (A_KC)
                As[(ak + e) * S::LDA + ar] = ra[e];
            else
                As[ak * S::LDA + ar + e] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < VB; ++e) {
            if constexpr (B_KC)
                Bs[(bk + e) * S::LDB + br] = rb[e];
            else
                Bs[bk * S::LDB + br + e] = rb[e];
        }
    };
    const int64_t nk = (K + S::BK - 1) / S::BK;
    if (nk <= 0)
        return;
    fa(ar, (int64_t)ak, ra);
    fb(br, (int64_t)bk, rb);
    store(lds, lds + S::A_ELEMS);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        double *cur = lds + (kt & 1) * S::STAGE;
        double *nxt = lds + ((kt + 1) & 1) * S::STAGE;
        const bool more = kt + 1 < nk;
        if (more) {
            fa(ar, (kt + 1) * S::BK + ak, ra);
            fb(br, (kt + 1) * S::BK + bk, rb);
        }
        mma_stage<S>(cur, cur + S::A_ELEMS, acc, wm, wn, lane);
        if (more)
            store(nxt, nxt + S::A_ELEMS);
        __syncthreads();
    }
}

// Same product with two loader pairs: faf / fbf for the full slices [0, K / BK)
// fill their run from a valid address without bounds checks and return true
// when it must be stored as zeros (applied at the store, after the stage's
// MFMAs); fa / fb (the checked run loaders above) load a ragged last slice,
// after the MFMAs of the stage before it.  With no branch on the loaded values
// in the loop, the next slice's loads stay in flight through the MFMAs.
template <class S, bool A_KC, bool B_KC, class FAF, class FBF, class FA, class FB>
DEV void gemm_tile_runs_ft(d4 (&acc)[S::FM][S::FN], double *lds, int64_t K, FAF faf, FBF fbf, FA fa, FB fb)
{
    constexpr int VA = S::BM * S::BK / S::NT;
    constexpr int VB = S::BN * S::BK / S::NT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave / S::WN, wn = wave % S::WN;
    double ra[VA], rb[VB];
    bool za = false, zb = false;
    int ar, ak, br, bk;
    if constexpr (A_KC) {
        ar = t / (S::BK / VA);
        ak = (t % (S::BK / VA)) * VA;
    } else {
        ak = t / (S::BM / VA);
        ar = (t % (S::BM / VA)) * VA;
    }
    if constexpr (B_KC) {
        br = t / (S::BK / VB);
        bk = (t % (S::BK / VB)) * VB;
    } else {
        bk = t / (S::BN / VB);
        br = (t % (S::BN / VB)) * VB;
    }
    auto store = [&](double *As, double *Bs) {
#pragma unroll
        for (int e = 0; e < VA; ++e) {
            const double v = za ? 0.0 : ra[e];
            if constexpr (A_KC)
                As[(ak + e) * S::LDA + ar] = v;
            else
                As[ak * S::LDA + ar + e] = v;
        }
#pragma unroll
        for (int e = 0; e < VB; ++e) {
            const double v = zb ? 0.0 : rb[e];
            if constexpr (B_KC)
                Bs[(bk + e) * S::LDB + br] = v;
            else
                Bs[bk * S::LDB + br + e] = v;
        }
    };
    const int64_t nk = (K + S::BK - 1) / S::BK, nkf = K / S::BK;
    if (nk <= 0)
        return;
    if (nkf > 0) {
        za = faf(ar, (int64_t)ak, ra);
        zb = fbf(br, (int64_t)bk, rb);
    } else {
        fa(ar, (int64_t)ak, ra);
        fb(br, (int64_t)bk, rb);
    }
    store(lds, lds + S::A_ELEMS);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        double *cur = lds + (kt & 1) * S::STAGE;
        double *nxt = lds + ((kt + 1) & 1) * S::STAGE;
        const bool more = kt + 1 < nkf;
        if (more) {
            za = faf(ar, (kt + 1) * S::BK + ak, ra);
            zb = fbf(br, (kt + 1) * S::BK + bk, rb);
        }
        mma_stage<S>(cur, cur + S::A_ELEMS, acc, wm, wn, lane);
        if (more) {
            store(nxt, nxt + S::A_ELEMS);
        } else if (kt + 1 < nk) {
            fa(ar, (kt + 1) * S::BK + ak, ra);
            fb(br, (kt + 1) * S::BK + bk, rb);
            za = zb = false;
            store(nxt, nxt + S::A_ELEMS);
        }
        __syncthreads();
    }
}

// Load n consecutive doubles from p (16-byte aligned when aligned16).
template <int N>
DEV void load_run(const double *__restrict__ p, double (&v)[N])
{
    static_assert(N % 2 == 0, "runs of an even length");
    const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int e = 0; e < N / 2; ++e) {
        const double2 x = q[e];
        v[2 * e] = x.x;
        v[2 * e + 1] = x.y;
    }
}

// ---------------------------------------------------------------------------
// FP32 MFMA tile machinery (v_mfma_f32_16x16x4_f32).  Operands are staged in
// LDS K-major as for FP64; lane l supplies A(l%16, l/16) and B(l/16, l%16);
// accumulator element e of lane l is C(4*(l/16) + e, l%16) (measured on
// gfx950).
// ---------------------------------------------------------------------------
template <class S>
DEV void zero_acc32(f4 (&acc)[S::FM][S::FN])
{
#pragma unroll
    for (int i = 0; i < S::FM; ++i)
#pragma unroll
        for (int j = 0; j < S::FN; ++j)
            acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
}

template <class S>
DEV void mma_stage32(const float *__restrict__ As, const float *__restrict__ Bs, f4 (&acc)[S::FM][S::FN],
                     int wm, int wn, int lane)
{
#pragma unroll
    for (int kk = 0; kk < S::BK; kk += 4) {
        const int kr = kk + (lane >> 4);
        float a[S::FM], b[S::FN];
#pragma unroll
        for (int i = 0; i < S::FM; ++i)
            a[i] = As[kr * S::LDA + wm * S::TM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < S::FN; ++j)
            b[j] = Bs[kr * S::LDB + wn * S::TN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < S::FM; ++i)
#pragma unroll
            for (int j = 0; j < S::FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

template <class S>
DEV int acc32_row(int wm, int i, int lane, int e) { return wm * S::TM + i * 16 + 4 * (lane >> 4) + e; }
template <class S>
DEV int acc32_col(int wn, int j, int lane, int e)
{
    (void)e;
    return wn * S::TN + j * 16 + (lane & 15);
}

// FP32 version of gemm_tile_runs (float LDS stages, same run-loader contract).
template <class S, bool A_KC, bool B_KC, class FA, class FB>
DEV void gemm_tile_runs32(f4 (&acc)[S::FM][S::FN], float *lds, int64_t K, FA fa, FB fb)
{
    constexpr int VA = S::BM * S::BK / S::NT;
    constexpr int VB = S::BN * S::BK / S::NT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave / S::WN, wn = wave % S::WN;
    float ra[VA], rb[VB];
    int ar, ak, br, bk;
    if constexpr (A_KC) {
        ar = t / (S::BK / VA);
        ak = (t % (S::BK / VA)) * VA;
    } else {
        ak = t / (S::BM / VA);
        ar = (t % (S::BM / VA)) * VA;
    }
    if constexpr (B_KC) {
        br = t / (S::BK / VB);
        bk = (t % (S::BK / VB)) * VB;
    } else {
        bk = t / (S::BN / VB);
        br = (t % (S::BN / VB)) * VB;
    }
    auto store = [&](float *As, float *Bs) {
#pragma unroll
        for (int e = 0; e < VA; ++e) {
            if constexpr (A_KC)
                As[(ak + e) * S::LDA + ar] = ra[e];
            else
                As[ak * S::LDA + ar + e] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < VB; ++e) {
            if constexpr (B_KC)
                Bs[(bk + e) * S::LDB + br] = rb[e];
            else
                Bs[bk * S::LDB + br + e] = rb[e];
        }
    };
    const int64_t nk = (K + S::BK - 1) / S::BK;
    if (nk <= 0)
        return;
    fa(ar, (int64_t)ak, ra);
    fb(br, (int64_t)bk, rb);
    store(lds, lds + S::A_ELEMS);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
        float *cur = lds + (kt & 1) * S::STAGE;
        float *nxt = lds + ((kt + 1) & 1) * S::STAGE;
        const bool more = kt + 1 < nk;
        if (more) {
            fa(ar, (kt + 1) * S::BK + ak, ra);
            fb(br, (kt + 1) * S::BK + bk, rb);
        }
        mma_stage32<S>(cur, cur + S::A_ELEMS, acc, wm, wn, lane);
        if (more)
            store(nxt, nxt + S::A_ELEMS);
        __syncthreads();
    }
}

// Load n consecutive floats (16-byte aligned).
template <int N>
DEV void load_run(const float *__restrict__ p, float (&v)[N])
{
    static_assert(N % 4 == 0, "runs of a multiple of 4 floats");
    const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int e = 0; e < N / 4; ++e) {
        const float4 x = q[e];
        v[4 * e] = x.x;
        v[4 * e + 1] = x.y;
        v[4 * e + 2] = x.z;
        v[4 * e + 3] = x.w;
    }
}
