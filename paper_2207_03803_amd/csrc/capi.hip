// C ABI of the GAP fit library: argument checks, workspace carving and the
// order in which the kernels are enqueued.  Declarations and the contract of
// each entry point are in include/gap.h.
#include <math.h>
#include <mutex>
#include <new>
#include <string.h>

#include "../../include/gap.h"
#include "kernels.h"

using namespace gap;

namespace {

constexpr int N_STAGES = 10;

enum State { ST_CREATED = 0, ST_BOUND = 1, ST_KNM = 2, ST_BUILT = 3, ST_SOLVED = 4 };

struct Layout {
    // N = all observation rows: NE energies (configurations) then n_obs derivative observations
    int64_t N = 0, M = 0, n_atoms = 0, m = 0, lda = 0, ncols = 0, max_tiles = 0;
    int64_t NE = 0, n_obs = 0, n_pos = 0, max_tiles_d = 0;
    size_t off_tiles_d = 0, off_plan_d = 0, off_D = 0;
    TsqrTree tree;
    size_t off_A = 0, off_tau = 0, off_wpart = 0, off_T = 0, off_Tin = 0, off_U = 0, off_W = 0, off_ts_tiles = 0,
           off_ts_X = 0, off_ts_tau = 0, off_rhs = 0, off_misc = 0, off_tiles = 0, off_counters = 0,
           off_status = 0, off_tflags = 0, n_tflags = 0, off_cq_S = 0, off_cq_part = 0, off_cq_G = 0, off_cq_R = 0,
           off_T2 = 0, off_wpart_s = 0, off_W_s = 0, off_W32_s = 0, off_plan = 0, total = 0;
    // mixed precision only
    bool mixed = false;
    size_t off_A32 = 0, off_W32 = 0, off_r = 0, off_s = 0, off_z = 0, off_dc = 0, off_p = 0, off_q = 0, off_part = 0,
           off_rnorm = 0, off_flags = 0, off_stats = 0;
    size_t off_diag = 0;  // diagnostics of the solution (eta, error estimate)
    // low-precision K_NM (GAP_MIXED_BF16 / GAP_MIXED_FP16) only: rounded descriptors
    bool lp = false;
    int dp = 0;
    size_t off_Xlp = 0, off_XMlp = 0;
    // INT8-emulated FP64 K_NM (GAP_FLAG_KNM_INT8) only: descriptor slices and row exponents
    bool oz = false;
    int dpo = 0;
    size_t off_Xoz = 0, off_XMoz = 0, off_xe = 0, off_xme = 0;
    // arrays GAP_FLAG_POISON_WORKSPACE fills (numbers and slices; no plans, counters or flags)
    static constexpr int MAX_POISON = 48;
    int n_poison = 0;
    size_t poison_off[MAX_POISON] = {}, poison_len[MAX_POISON] = {};
};

bool is_mixed(int32_t precision) { return precision != GAP_FP64; }
bool is_lp(int32_t precision) { return precision == GAP_MIXED_BF16 || precision == GAP_MIXED_FP16; }

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

Layout make_layout(int64_t NE, int64_t n_atoms, int64_t M, int32_t precision, int d, uint32_t flags,
                   int64_t n_obs = 0, int64_t n_pos = 0)
{
    Layout L;
    const int64_t N = NE + n_obs;
    L.NE = NE;
    L.n_obs = n_obs;
    L.n_pos = n_pos;
    const bool mixed = is_mixed(precision);
    L.mixed = mixed;
    L.lp = is_lp(precision);
    L.N = N;
    L.M = M;
    L.n_atoms = n_atoms;
    L.m = N + M;
    L.lda = (L.m + 63) / 64 * 64;
    L.ncols = M + 1;
    L.max_tiles = knm_max_tiles(NE, n_atoms);
    L.tree = tsqr_tree(L.m);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    auto takep = [&](size_t bytes) {  // a numeric array: filled under GAP_FLAG_POISON_WORKSPACE
        const size_t at = take(bytes);
        if (L.n_poison < Layout::MAX_POISON) {
            L.poison_off[L.n_poison] = at;
            L.poison_len[L.n_poison++] = bytes;
        }
        return at;
    };
    L.off_A = takep(sizeof(double) * (size_t)L.lda * (size_t)L.ncols);
    L.off_tau = takep(sizeof(double) * (size_t)M);
    L.off_wpart = takep(sizeof(double) * (size_t)qr_max_chunks() * 4 * QR_NB * (size_t)L.ncols);
    L.off_T = takep(sizeof(double) * 16 * QR_NB * QR_NB);
    L.off_Tin = takep(sizeof(double) * 2 * QR_NB * QR_NB);
    L.off_U = takep(sizeof(double) * QR_NB * QR_NB);
    L.off_W = takep(sizeof(double) * 4 * QR_NB * (size_t)((L.ncols + 63) / 64 * 64));
    L.off_ts_tiles = takep(sizeof(double) * (size_t)L.tree.tiles_doubles);
    L.off_ts_X = takep(sizeof(double) * (size_t)L.tree.tiles_doubles);
    L.off_ts_tau = takep(sizeof(double) * (size_t)L.tree.tau_doubles);
    L.off_rhs = takep(sizeof(double) * (size_t)M);
    L.off_misc = takep(sizeof(double) * 512);
    L.off_tiles = take(sizeof(int32_t) * (size_t)(L.max_tiles + 2));
    L.off_plan = take(sizeof(int32_t) * (size_t)(NE + knm_plan_chunks(NE) * (2049 + 1)));
    if (n_obs > 0) {
        // derivative observations: their tile plan over the positions, and D = (X X_M^T)^(zeta - 1)
        L.max_tiles_d = knm_max_tiles(n_obs, n_pos);
        L.off_tiles_d = take(sizeof(int32_t) * (size_t)(L.max_tiles_d + 2));
        L.off_plan_d = take(sizeof(int32_t) * (size_t)(n_obs + knm_plan_chunks(n_obs) * (2049 + 1)));
        L.off_D = takep(sizeof(double) * (size_t)n_atoms * (size_t)M);
    }
    L.off_counters = take(sizeof(unsigned) * 16);
    L.off_status = take(sizeof(int32_t) * 4);
    L.n_tflags = trsv_sync_ints(M);
    L.off_tflags = take(sizeof(int32_t) * (size_t)L.n_tflags);
    L.off_cq_S = takep(sizeof(double) * QR_NB * (size_t)L.lda);
    L.off_cq_part = takep(sizeof(double) * (size_t)CQ_MAX_CHUNKS * QR_NB * QR_NB);
    L.off_cq_G = takep(sizeof(double) * 4 * QR_NB * QR_NB);
    L.off_cq_R = takep(sizeof(double) * 4 * QR_NB * QR_NB);
    L.off_T2 = takep(sizeof(double) * 16 * QR_NB * QR_NB);
    L.off_wpart_s = takep(sizeof(double) * (size_t)qr_max_chunks_s() * 4 * QR_NB * 2 * QR_NB);
    L.off_W_s = takep(sizeof(double) * 16 * QR_NB * QR_NB);
    L.off_W32_s = takep(sizeof(float) * 16 * QR_NB * QR_NB);
    L.off_diag = takep(sizeof(double) * (size_t)(14 * M + 512));
    if (mixed) {
        const int64_t ldw = (L.ncols + 63) / 64 * 64;
        L.off_A32 = takep(sizeof(float) * (size_t)L.lda * (size_t)L.ncols);
        L.off_W32 = takep(sizeof(float) * 4 * QR_NB * (size_t)ldw);
        L.off_r = takep(sizeof(double) * (size_t)L.m);
        L.off_s = takep(sizeof(double) * (size_t)M);
        L.off_z = takep(sizeof(double) * (size_t)M);
        L.off_dc = takep(sizeof(double) * (size_t)M);
        L.off_p = takep(sizeof(double) * (size_t)M);
        L.off_q = takep(sizeof(double) * (size_t)L.m);
        L.off_part = takep(sizeof(double) * 8 * (size_t)L.m);
        L.off_rnorm = takep(sizeof(double) * (size_t)((L.m + 255) / 256 + 1));
        L.off_flags = take(sizeof(int32_t) * 4);
        L.off_stats = takep(sizeof(double) * 4);
    }
    if (L.lp) {
        L.dp = knm_lp_dpad(d);
        L.off_Xlp = takep(sizeof(uint16_t) * (size_t)n_atoms * (size_t)L.dp);
        L.off_XMlp = takep(sizeof(uint16_t) * (size_t)M * (size_t)L.dp);
    }
    if (flags & GAP_FLAG_KNM_INT8) {
        L.oz = true;
        L.dpo = knm_oz_dpad(d);
        const size_t sl = (size_t)knm_oz_slices();
        L.off_Xoz = takep(sl * (size_t)n_atoms * (size_t)L.dpo);
        L.off_XMoz = takep(sl * (size_t)M * (size_t)L.dpo);
        L.off_xe = takep(sizeof(int32_t) * (size_t)n_atoms);
        L.off_xme = takep(sizeof(int32_t) * (size_t)M);
    }
    L.total = o;
    return L;
}

}  // namespace

struct gap_handle_s {
    gap_params p;
    hipStream_t stream = nullptr;
    int device = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int state = ST_CREATED;
    Layout L;
    const double *x_sparse = nullptr;
    const double *sigma = nullptr;
    const double *x_atoms = nullptr;      // inputs of the current build
    const int64_t *offsets = nullptr;
    gap_deriv_obs obs = {};   // derivative observations of the current build (n_obs = 0: none)
    int64_t model_M = 0;      // set by gap_set_model
    bool model_only = false;  // predict-only handle (no workspace)
    hipEvent_t ev[2 * N_STAGES] = {};
    QrAsync la = {};   // side stream and events of the QR look-ahead
    int la_free_cus = 0;  // CUs the side stream was created without
    bool timed[N_STAGES] = {};
    bool timing = false;
    gap_tuning tuning = {};

    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    double *A() const { return at<double>(L.off_A); }
    int32_t *status() const { return at<int32_t>(L.off_status); }
    unsigned *counters() const { return at<unsigned>(L.off_counters); }
    double *misc() const { return at<double>(L.off_misc); }
    // flags of the one-launch triangular solves; counters()[12] is their arrival counter
    TrsvSync tsync() const { return TrsvSync{at<int32_t>(L.off_tflags), counters() + 12, status()}; }

    // diagnostics area: [8M] partials, partR, t, g, x, y, z [M each], sc[4], sumsq partials[256], out[4]
    DiagWork diag(double *g_override) const
    {
        double *base = at<double>(L.off_diag);
        const int64_t M = L.M;
        DiagWork d{};
        d.n = M;
        d.ld = L.lda;
        d.part = base;
        d.partR = base + 8 * M;
        d.t = base + 9 * M;
        d.g = g_override ? g_override : base + 10 * M;
        d.x = base + 11 * M;
        d.y = base + 12 * M;
        d.z = base + 13 * M;
        d.sc = base + 14 * M;
        d.sum_part = d.sc + 4;
        d.counter = counters() + 9;
        d.tail2 = misc();
        d.iters = (p.flags & GAP_FLAG_ERROR_ESTIMATE) ? 16 : 0;
        d.sync = tsync();
        return d;
    }
    double *diag_out() const { return at<double>(L.off_diag) + 14 * L.M + 4 + 256; }

    void mark_on(int stage, bool end, hipStream_t st)
    {
        if (!timing)
            return;
        (void)hipEventRecord(ev[2 * stage + (end ? 1 : 0)], st);
        if (end)
            timed[stage] = true;
    }
    void mark(int stage, bool end) { mark_on(stage, end, stream); }
};

namespace {

__global__ void zero_u32_kernel(unsigned *p, int n)
{
    if ((int)threadIdx.x < n)
        p[threadIdx.x] = 0u;
}

__global__ void zero_i32_kernel(int32_t *p, int64_t n)
{
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        p[i] = 0;
}

// All-ones words over n 4-byte words (GAP_FLAG_POISON_WORKSPACE).
__global__ void poison_kernel(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0xFFFFFFFFu;
}

__global__ void copy_kernel(const double *src, double *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        dst[i] = src[i];
}

// Where gap_predict reports malformed offsets: the fit's status word, or, on a
// predict-only handle, the first word of a bound workspace (none without one).
int32_t *predict_status(gap_handle h)
{
    if (!h->ws)
        return nullptr;
    return h->model_only ? reinterpret_cast<int32_t *>(h->ws) : h->status();
}

bool valid_params(const gap_params *p)
{
    // the INT8-emulated K_NM sums at most 7 slice products of d_pad terms of up to 2^14
    // exactly in INT32 only for d_pad <= 4096
    if (p && (p->flags & GAP_FLAG_KNM_INT8) && knm_oz_dpad(p->d) > 4096)
        return false;
    return p && p->d >= 1 && p->zeta >= 1 && p->zeta <= 8 && p->sigma_w > 0.0 && isfinite(p->sigma_w) &&
           p->jitter >= 0.0 && isfinite(p->jitter) &&
           (p->precision == GAP_FP64 || p->precision == GAP_MIXED_FP32 || p->precision == GAP_MIXED_BF16 ||
            p->precision == GAP_MIXED_FP16) &&
           (p->precision == GAP_FP64 || (p->max_refine_iters >= 0 && p->max_refine_iters <= 1000 &&
                                          p->refine_tol >= 0.0));
}

gap_status dev(hipError_t e) { return e == hipSuccess ? GAP_OK : GAP_EDEVICE; }

#define GAP_TRY(expr)                      \
    do {                                   \
        gap_status s_ = (expr);            \
        if (s_ != GAP_OK)                  \
            return s_;                     \
    } while (0)

}  // namespace

extern "C" {

size_t gap_cur_workspace_bytes(int64_t n_rows, int32_t d)
{
    if (n_rows < 1 || d < 1 || d > cur_max_d() || n_rows < d)
        return 0;
    return cur_workspace_bytes(n_rows, d);
}

gap_status gap_cur_select(const double *x, int64_t n_rows, int32_t d, const double *exp_draws, int64_t M,
                          int64_t *selected, double *leverage, void *workspace, size_t workspace_bytes,
                          void *stream, int32_t wait)
{
    if (!x || !selected || !workspace || d < 1 || d > cur_max_d() || n_rows < d || M < 1 || M > n_rows)
        return GAP_EINVAL;
    if (workspace_bytes < cur_workspace_bytes(n_rows, d))
        return GAP_ENOMEM;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    CurLaunch c{};
    c.x = x;
    c.n = n_rows;
    c.d = d;
    c.draws = exp_draws;
    c.M = M;
    c.out = selected;
    c.lev_out = leverage;
    c.workspace = workspace;
    if (launch_cur_select(c, s) != hipSuccess)
        return GAP_EDEVICE;
    if (!wait)
        return GAP_OK;
    int32_t st = 0;
    if (hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(&st, static_cast<char *>(workspace) + cur_status_offset(), sizeof(st), hipMemcpyDeviceToHost) !=
            hipSuccess)
        return GAP_EDEVICE;
    return st == 0 ? GAP_OK : static_cast<gap_status>(st);
}

const char *gap_status_string(gap_status s)
{
    switch (s) {
    case GAP_OK: return "ok";
    case GAP_EINVAL: return "invalid argument";
    case GAP_ENOMEM: return "workspace too small";
    case GAP_ENOTPD: return "K_MM + jitter is not positive definite";
    case GAP_ENONFINITE: return "non-finite value in the weights";
    case GAP_ENOCONV: return "refinement did not converge";
    case GAP_ERANK: return "stacked matrix numerically rank deficient";
    case GAP_EDEVICE: return "HIP runtime error";
    case GAP_ESTATE: return "entry point called out of order";
    }
    return "unknown status";
}

size_t gap_workspace_bytes(const gap_params *p, int64_t n_configs, int64_t n_atoms, int64_t M)
{
    if (!valid_params(p) || n_configs < 1 || n_atoms < 0 || M < 1)
        return 0;
    return make_layout(n_configs, n_atoms, M, p->precision, p->d, p->flags).total;
}

// Release a handle's events and side stream (those created so far) and the handle.
static void destroy_handle(gap_handle h)
{
    for (int i = 0; i < 2 * N_STAGES; ++i)
        if (h->ev[i])
            (void)hipEventDestroy(h->ev[i]);
    hipEvent_t lev[5] = {h->la.fork, h->la.t_ready, h->la.bulk[0], h->la.bulk[1], h->la.join};
    for (hipEvent_t e : lev)
        if (e)
            (void)hipEventDestroy(e);
    if (h->la.side)
        (void)hipStreamDestroy(h->la.side);
    delete h;
}

gap_status gap_create(const gap_params *p, void *stream, gap_handle *out)
{
    if (!out || !valid_params(p))
        return GAP_EINVAL;
    *out = nullptr;
    gap_handle h = new (std::nothrow) gap_handle_s();
    if (!h)
        return GAP_EDEVICE;
    h->p = *p;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    h->timing = (p->flags & GAP_FLAG_TIMING) != 0;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return GAP_EDEVICE;
    }
    if (h->timing) {
        for (int i = 0; i < 2 * N_STAGES; ++i)
            if (hipEventCreate(&h->ev[i]) != hipSuccess) {
                destroy_handle(h);
                return GAP_EDEVICE;
            }
    }

    *out = h;
    return GAP_OK;
}

gap_status gap_bind_workspace(gap_handle h, void *dev_ptr, size_t bytes)
{
    if (!h || !dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255u))
        return GAP_EINVAL;
    if (h->model_only && bytes < 16)
        return GAP_EINVAL;
    h->ws = static_cast<char *>(dev_ptr);
    h->ws_bytes = bytes;
    h->state = ST_BOUND;
    if (h->model_only) {
        // a predict-only handle keeps its status word in the workspace's first bytes
        hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, h->stream, reinterpret_cast<unsigned *>(h->ws), 4);
        return dev(hipGetLastError());
    }
    return GAP_OK;
}

// Look-ahead pays where the panels are many: automatic from 2048 columns on.
static bool use_lookahead(gap_handle h)
{
    const int32_t mode = h->tuning.qr_lookahead;
    return mode == 2 || (mode == 0 && h->L.M >= 2048);
}

// The look-ahead's stream and events, created the first time a fit needs them.
// CUs kept free of the look-ahead stream (0: an unmasked stream).  Opt-in: a
// masked stream is a blocking one, which serialises with any work on the
// legacy default stream, e.g. other threads' copies in a serving loop.
static int free_cus_for(gap_handle h) { return h->tuning.qr_free_cus; }

// The look-ahead stream.  With free CUs it is created with a CU mask that
// leaves them to the handle's stream (the panel chain of the next block); such
// a stream is a blocking one, so it also orders itself with the legacy default
// stream.
static bool create_lookahead(gap_handle h)
{
    const int freecus = free_cus_for(h);
    hipError_t e0 = hipSuccess;
    if (freecus > 0) {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || ncu < 1)
            return false;
        const int words = (ncu + 31) / 32;
        uint32_t mask[64] = {};
        if (words > 64 || freecus >= ncu)
            return false;
        for (int c = freecus; c < ncu; ++c)
            mask[c / 32] |= 1u << (c % 32);
        e0 = hipExtStreamCreateWithCUMask(&h->la.side, (uint32_t)words, mask);
    } else {
        e0 = hipStreamCreateWithFlags(&h->la.side, hipStreamNonBlocking);
    }
    if (e0 != hipSuccess) {
        h->la.side = nullptr;
        return false;
    }
    h->la_free_cus = freecus;
    hipEvent_t *lev[5] = {&h->la.fork, &h->la.t_ready, &h->la.bulk[0], &h->la.bulk[1], &h->la.join};
    for (hipEvent_t *e : lev)
        if (!*e && hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
            *e = nullptr;
            return false;  // the handle keeps what was created; gap_destroy releases it
        }
    return true;
}

// Checks, layout and input pointers of a build; creates the look-ahead stream
// when the fit uses one.
static gap_status build_prepare(gap_handle h, const double *x_atoms, int64_t n_atoms, const int64_t *config_offsets,
                                int64_t n_configs, const double *x_sparse, int64_t M, const double *sigma,
                                const gap_deriv_obs *obs = nullptr)
{
    if (!h)
        return GAP_EINVAL;
    if (h->state < ST_BOUND)
        return GAP_ESTATE;
    if (!x_atoms || !config_offsets || !x_sparse || !sigma || n_atoms < 1 || n_configs < 1 || M < 1 ||
        n_configs > INT32_MAX - 1)
        return GAP_EINVAL;
    if (obs && (!obs->x_grad || !obs->grad_atom || !obs->obs_offsets || !obs->pos_grad || !obs->pos_weight ||
                obs->n_grad < 1 || obs->n_obs < 1 || obs->n_pos < 1 || is_lp(h->p.precision)))
        return GAP_EINVAL;
    const Layout L = make_layout(n_configs, n_atoms, M, h->p.precision, h->p.d, h->p.flags, obs ? obs->n_obs : 0,
                                 obs ? obs->n_pos : 0);
    if (L.total > h->ws_bytes)
        return GAP_ENOMEM;
    h->L = L;
    h->obs = obs ? *obs : gap_deriv_obs{};
    h->timed[9] = false;
    h->x_atoms = x_atoms;
    h->offsets = config_offsets;
    h->x_sparse = x_sparse;
    h->sigma = sigma;
    h->model_only = false;
    if (use_lookahead(h) && h->la.side && h->la_free_cus != free_cus_for(h)) {
        // the CU mask changed: replace the stream (after its last work)
        if (hipStreamSynchronize(h->la.side) != hipSuccess || hipStreamDestroy(h->la.side) != hipSuccess)
            return GAP_EDEVICE;
        h->la.side = nullptr;
    }
    if (use_lookahead(h) && !h->la.side && !create_lookahead(h))
        return GAP_EDEVICE;
    return GAP_OK;
}

static KnmPlan plan_of(gap_handle h)
{
    const Layout &L = h->L;
    int32_t *tiles = h->at<int32_t>(L.off_tiles);
    int32_t *plan = h->at<int32_t>(L.off_plan);
    KnmPlan kp;
    kp.tile_start = tiles;
    kp.n_tiles = tiles + L.max_tiles + 1;
    kp.cfg_list = plan;
    kp.lstart = plan + L.NE;
    kp.lcount = kp.lstart + knm_plan_chunks(L.NE) * 2049;
    return kp;
}

// The derivative observations' tile plan (over their positions).
static KnmPlan plan_of_d(gap_handle h)
{
    const Layout &L = h->L;
    int32_t *tiles = h->at<int32_t>(L.off_tiles_d);
    int32_t *plan = h->at<int32_t>(L.off_plan_d);
    KnmPlan kp;
    kp.tile_start = tiles;
    kp.n_tiles = tiles + L.max_tiles_d + 1;
    kp.cfg_list = plan;
    kp.lstart = plan + L.n_obs;
    kp.lcount = kp.lstart + knm_plan_chunks(L.n_obs) * 2049;
    return kp;
}

// On stream s: clear the counters, status and flags, and plan the K_NM tiles;
// *a = the fit's K_NM launch arguments.
static gap_status build_setup(gap_handle h, hipStream_t s, KnmArgs *a)
{
    const Layout &L = h->L;
    if (h->p.flags & GAP_FLAG_POISON_WORKSPACE)
        for (int i = 0; i < L.n_poison; ++i) {
            // each array starts 256-byte aligned and its padding runs to the next multiple of 256
            const int64_t words = (int64_t)((L.poison_len[i] + 3) / 4);
            if (words == 0)
                continue;
            const unsigned blocks = (unsigned)std::min<int64_t>((words + 255) / 256, 4096);
            hipLaunchKernelGGL(poison_kernel, dim3(blocks), dim3(256), 0, s, h->at<uint32_t>(L.poison_off[i]), words);
        }
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, h->counters(), 16);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned *>(h->status()), 4);
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(256), 0, s, h->at<int32_t>(L.off_tflags), L.n_tflags);
    const KnmPlan kp = plan_of(h);
    GAP_TRY(dev(launch_plan_tiles(h->offsets, L.NE, L.n_atoms, kp, L.max_tiles, h->status(), s)));
    *a = KnmArgs{};
    a->X = h->x_atoms;
    a->offsets = h->offsets;
    a->tile_start = kp.tile_start;
    a->cfg_list = kp.cfg_list;
    a->n_tiles_dev = kp.n_tiles;
    a->XM = h->x_sparse;
    a->M = L.M;
    a->d = h->p.d;
    a->zeta = h->p.zeta;
    a->sw2 = h->p.sigma_w * h->p.sigma_w;
    a->sigma = h->sigma;
    a->out = h->A();
    a->ldo = L.lda;
    a->row_off = 0;
    a->status = h->status();
    a->bn = h->tuning.knm_bn;
    return GAP_OK;
}

// The FP64 K_NM from INT8 slice products (GAP_FLAG_KNM_INT8), after build_setup's plan.
static gap_status launch_knm_int8(gap_handle h, hipStream_t s)
{
    const Layout &L = h->L;
    const gap_params &p = h->p;
    int8_t *Xoz = h->at<int8_t>(L.off_Xoz), *XMoz = h->at<int8_t>(L.off_XMoz);
    int32_t *xe = h->at<int32_t>(L.off_xe), *xme = h->at<int32_t>(L.off_xme);
    GAP_TRY(dev(launch_oz_split(h->x_atoms, L.n_atoms, p.d, Xoz, xe, s)));
    GAP_TRY(dev(launch_oz_split(h->x_sparse, L.M, p.d, XMoz, xme, s)));
    const KnmPlan kp = plan_of(h);
    KnmOzLaunch l{};
    l.X = Xoz;
    l.XM = XMoz;
    l.xe = xe;
    l.xme = xme;
    l.n_atoms = L.n_atoms;
    l.d = p.d;
    l.offsets = h->offsets;
    l.tile_start = kp.tile_start;
    l.cfg_list = kp.cfg_list;
    l.n_tiles_dev = kp.n_tiles;
    l.max_tiles = L.max_tiles;
    l.M = L.M;
    l.zeta = p.zeta;
    l.sw2 = p.sigma_w * p.sigma_w;
    l.sigma = h->sigma;
    l.out = h->A();
    l.ldo = L.lda;
    return dev(launch_knm_oz(l, s));
}

// On the handle's stream, after the K_NM: the low-precision K_NM (mixed BF16 /
// FP16), K_MM + jitter (upper triangle) into rows N..N+M-1, then U = L^T in place.
// K_MM + jitter and its Cholesky into the bottom block of A, on stream s.
static gap_status launch_kmm_chol(gap_handle h, hipStream_t s)
{
    const Layout &L = h->L;
    const gap_params &p = h->p;
    KnmArgs k{};
    k.X = h->x_sparse;
    k.offsets = nullptr;
    k.n_rows_unit = L.M;
    k.XM = h->x_sparse;
    k.M = L.M;
    k.d = p.d;
    k.zeta = p.zeta;
    k.sw2 = p.sigma_w * p.sigma_w;
    k.sigma = nullptr;
    k.out = h->A();
    k.ldo = L.lda;
    k.row_off = L.N;
    k.jitter = p.jitter;
    k.upper_only = 1;
    k.status = h->status();
    h->mark_on(1, false, s);
    GAP_TRY(dev(launch_knm(k, (L.M + KNM_BM - 1) / KNM_BM, s)));
    h->mark_on(1, true, s);
    h->mark_on(2, false, s);
    GAP_TRY(dev(launch_potrf_upper(h->A() + L.N, L.lda, L.M, h->status(), s)));
    h->mark_on(2, true, s);
    return GAP_OK;
}

// K_MM and its Cholesky need neither the K_NM nor its plan: with a look-ahead stream
// they run there, beside the K_NM (forked after the build's set-up, joined in
// build_rest); without one build_rest runs them in order.
static gap_status fork_kmm(gap_handle h, bool &forked)
{
    forked = false;
    if (!h->la.side || !h->la.fork || !h->la.join)
        return GAP_OK;
    if (hipEventRecord(h->la.fork, h->stream) != hipSuccess ||
        hipStreamWaitEvent(h->la.side, h->la.fork, 0) != hipSuccess)
        return GAP_EDEVICE;
    GAP_TRY(launch_kmm_chol(h, h->la.side));
    if (hipEventRecord(h->la.join, h->la.side) != hipSuccess)
        return GAP_EDEVICE;
    forked = true;
    return GAP_OK;
}

static gap_status build_rest(gap_handle h, bool kmm_forked = false)
{
    const Layout &L = h->L;
    hipStream_t s = h->stream;
    const gap_params &p = h->p;
    const double sw2 = p.sigma_w * p.sigma_w;
    if (L.lp) {
        // the factor's copy of Sigma^-1/2 K_NM from BF16 / FP16 dot products (FP32 power and sums)
        const bool bf = p.precision == GAP_MIXED_BF16;
        uint16_t *Xlp = h->at<uint16_t>(L.off_Xlp), *XMlp = h->at<uint16_t>(L.off_XMlp);
        const KnmPlan kp = plan_of(h);
        h->mark(7, false);
        GAP_TRY(dev(launch_convert_lp(h->x_atoms, L.n_atoms, p.d, Xlp, bf, s)));
        GAP_TRY(dev(launch_convert_lp(h->x_sparse, L.M, p.d, XMlp, bf, s)));
        KnmLpLaunch l{};
        l.X = Xlp;
        l.XM = XMlp;
        l.d = p.d;
        l.offsets = h->offsets;
        l.tile_start = kp.tile_start;
        l.cfg_list = kp.cfg_list;
        l.n_tiles_dev = kp.n_tiles;
        l.max_tiles = L.max_tiles;
        l.M = L.M;
        l.zeta = p.zeta;
        l.sw2 = sw2;
        l.sigma = h->sigma;
        l.out = h->at<float>(L.off_A32);
        l.ldo = L.lda;
        l.bf16 = bf;
        GAP_TRY(dev(launch_knm_lp(l, s)));
        h->mark(7, true);
    }
    if (kmm_forked) {
        if (hipStreamWaitEvent(s, h->la.join, 0) != hipSuccess)
            return GAP_EDEVICE;
    } else {
        GAP_TRY(launch_kmm_chol(h, s));
    }
    h->state = ST_BUILT;
    return GAP_OK;
}

gap_status gap_build_knm(gap_handle h, const double *x_atoms, int64_t n_atoms, const int64_t *config_offsets,
                         int64_t n_configs, const double *x_sparse, int64_t M, const double *sigma)
{
    GAP_TRY(build_prepare(h, x_atoms, n_atoms, config_offsets, n_configs, x_sparse, M, sigma));
    KnmArgs a;
    GAP_TRY(build_setup(h, h->stream, &a));
    bool forked = false;
    GAP_TRY(fork_kmm(h, forked));
    h->mark(0, false);
    if (h->L.oz)
        GAP_TRY(launch_knm_int8(h, h->stream));
    else
        GAP_TRY(dev(launch_knm(a, h->L.max_tiles, h->stream)));
    h->mark(0, true);
    return build_rest(h, forked);
}

// Derivative observation rows N_E .. N_E + n_obs - 1 of A: D = (X X_M^T)^(zeta - 1) for
// every atom (none for zeta = 1), the positions' tile plan, then the derivative tiles.
static gap_status build_derivatives(gap_handle h)
{
    const Layout &L = h->L;
    const gap_params &p = h->p;
    hipStream_t s = h->stream;
    const gap_deriv_obs &o = h->obs;
    h->mark(9, false);
    double *D = nullptr;
    if (p.zeta > 1) {
        // row-major D[i * M + j]: the sparse points as the unit rows and the atoms as the
        // columns of the column-major output, so that a position's row of D is contiguous
        D = h->at<double>(L.off_D);
        KnmArgs k{};
        k.X = h->x_sparse;
        k.offsets = nullptr;
        k.n_rows_unit = L.M;
        k.XM = h->x_atoms;
        k.M = L.n_atoms;
        k.d = p.d;
        k.zeta = p.zeta - 1;
        k.sw2 = 1.0;
        k.out = D;
        k.ldo = L.M;
        k.status = h->status();
        GAP_TRY(dev(launch_knm(k, (L.M + KNM_BM - 1) / KNM_BM, s)));
    }
    const KnmPlan kp = plan_of_d(h);
    GAP_TRY(dev(launch_plan_tiles(o.obs_offsets, L.n_obs, L.n_pos, kp, L.max_tiles_d, h->status(), s)));
    KnmArgs a{};
    a.X = o.x_grad;
    a.offsets = o.obs_offsets;
    a.tile_start = kp.tile_start;
    a.cfg_list = kp.cfg_list;
    a.n_tiles_dev = kp.n_tiles;
    a.XM = h->x_sparse;
    a.M = L.M;
    a.d = p.d;
    a.zeta = p.zeta;
    a.sw2 = p.sigma_w * p.sigma_w;
    a.sigma = h->sigma + L.NE;
    a.out = h->A();
    a.ldo = L.lda;
    a.row_off = L.NE;
    a.status = h->status();
    a.pos_grad = o.pos_grad;
    a.pos_weight = o.pos_weight;
    a.grad_atom = o.grad_atom;
    a.D = D;
    a.ldd = L.M;
    a.n_grad = o.n_grad;
    a.n_src = L.n_atoms;
    GAP_TRY(dev(launch_kdm(a, L.max_tiles_d, s)));
    h->mark(9, true);
    return GAP_OK;
}

gap_status gap_build_knm_obs(gap_handle h, const double *x_atoms, int64_t n_atoms, const int64_t *config_offsets,
                             int64_t n_configs, const gap_deriv_obs *obs, const double *x_sparse, int64_t M,
                             const double *sigma)
{
    if (!obs)
        return GAP_EINVAL;
    GAP_TRY(build_prepare(h, x_atoms, n_atoms, config_offsets, n_configs, x_sparse, M, sigma, obs));
    KnmArgs a;
    GAP_TRY(build_setup(h, h->stream, &a));
    bool forked = false;
    GAP_TRY(fork_kmm(h, forked));
    h->mark(0, false);
    if (h->L.oz)
        GAP_TRY(launch_knm_int8(h, h->stream));
    else
        GAP_TRY(dev(launch_knm(a, h->L.max_tiles, h->stream)));
    h->mark(0, true);
    GAP_TRY(build_derivatives(h));
    return build_rest(h, forked);
}

size_t gap_workspace_bytes_obs(const gap_params *p, int64_t n_configs, int64_t n_atoms, int64_t n_obs,
                               int64_t n_pos, int64_t M)
{
    if (!valid_params(p) || n_configs < 1 || n_atoms < 1 || M < 1 || n_obs < 0 || n_pos < 0 ||
        (n_obs > 0 && n_pos < 1) || n_configs + n_obs > INT32_MAX - 1 || n_obs > INT32_MAX - 1)
        return 0;
    return make_layout(n_configs, n_atoms, M, p->precision, p->d, p->flags, n_obs, n_pos).total;
}

gap_status gap_build_knm_batch(gap_handle *handles, int32_t n, const gap_batch_fit *fits, void *stream)
{
    if (!handles || !fits || n < 1 || n > 4096)
        return GAP_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (int32_t i = 0; i < n; ++i) {
        const gap_batch_fit &f = fits[i];
        GAP_TRY(build_prepare(handles[i], f.x_atoms, f.n_atoms, f.config_offsets, f.n_configs, f.x_sparse, f.M,
                              f.sigma));
        for (int32_t j = 0; j < i; ++j)
            if (handles[j] == handles[i])
                return GAP_EINVAL;
    }
    // FP64-MFMA fits in groups of up to KNM_GROUP per launch; INT8-emulated ones launch alone
    KnmArgs args[KNM_GROUP];
    int64_t max_tiles[KNM_GROUP];
    int g = 0;
    for (int32_t i = 0; i < n; ++i) {
        gap_handle hi = handles[i];
        GAP_TRY(build_setup(hi, s, &args[g]));
        if (hi->L.oz) {
            GAP_TRY(launch_knm_int8(hi, s));
            continue;
        }
        max_tiles[g] = hi->L.max_tiles;
        if (++g == KNM_GROUP) {
            GAP_TRY(dev(launch_knm_group(args, max_tiles, g, s)));
            g = 0;
        }
    }
    if (g > 0)
        GAP_TRY(dev(launch_knm_group(args, max_tiles, g, s)));
    for (int32_t i = 0; i < n; ++i) {
        handles[i]->timed[0] = false;
        handles[i]->state = ST_KNM;
    }
    return GAP_OK;
}

gap_status gap_build_kmm(gap_handle h)
{
    if (!h)
        return GAP_EINVAL;
    if (h->state != ST_KNM)
        return GAP_ESTATE;
    return build_rest(h);
}

gap_status gap_sync(gap_handle h, gap_solve_info *info)
{
    if (!h)
        return GAP_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess)
        return GAP_EDEVICE;
    int32_t st = 0;
    double res = 0.0;
    if (h->model_only && h->ws) {
        if (hipMemcpy(&st, h->ws, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
            return GAP_EDEVICE;
    } else if (h->ws && h->L.total) {
        if (hipMemcpy(&st, h->status(), sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
            return GAP_EDEVICE;
        if (hipMemcpy(&res, h->misc(), sizeof(res), hipMemcpyDeviceToHost) != hipSuccess)
            return GAP_EDEVICE;
    }
    if (info) {
        memset(info, 0, sizeof(*info));
        info->device_status = st;
        info->residual_norm2 = res;
        if (h->ws && h->L.total && h->L.mixed) {
            int32_t it[2] = {0, 0};
            double st2[2] = {0.0, 0.0};
            if (hipMemcpy(it, h->at<int32_t>(h->L.off_flags) + 1, sizeof(it), hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(st2, h->at<double>(h->L.off_stats), sizeof(st2), hipMemcpyDeviceToHost) != hipSuccess)
                return GAP_EDEVICE;
            info->refine_iters = it[0];
            info->cgls_iters = it[1];
            info->step_rel = st2[1];
        }
        if (h->ws && h->L.total && h->state == ST_SOLVED) {
            double dg[3] = {0.0, -1.0, 0.0};
            if (hipMemcpy(dg, h->diag_out(), sizeof(dg), hipMemcpyDeviceToHost) != hipSuccess)
                return GAP_EDEVICE;
            info->grad_rel = dg[0];
            info->est_err = dg[1];
            info->kappa_est = dg[1] >= 0.0 ? dg[2] : 0.0;
        } else {
            info->est_err = -1.0;
        }
    }
    return (gap_status)st;
}

gap_status gap_solve(gap_handle h, const double *y, double *c_out, gap_solve_info *info)
{
    if (!h || !y || !c_out)
        return GAP_EINVAL;
    if (h->state != ST_BUILT)
        return GAP_ESTATE;
    const Layout &L = h->L;
    hipStream_t s = h->stream;
    double *A = h->A();
    h->mark(3, false);
    GAP_TRY(dev(launch_assemble_b(y, h->sigma, L.N, A + L.M * L.lda, L.lda, s)));
    h->mark(3, true);

    QrWork w{};
    w.A = A;
    w.lda = L.lda;
    w.m = L.m;
    w.tri0 = L.N;  // rows N.. hold L^T, upper triangular
    w.n = L.M;
    w.ncols = L.ncols;
    w.ldw = (L.ncols + 63) / 64 * 64;
    w.wp_ld = L.ncols;
    w.T2 = h->at<double>(L.off_T2);
    w.wpart_s = h->at<double>(L.off_wpart_s);
    w.W_s = h->at<double>(L.off_W_s);
    w.W32_s = h->at<float>(L.off_W32_s);
    w.tau = h->at<double>(L.off_tau);
    w.wpart = h->at<double>(L.off_wpart);
    w.T = h->at<double>(L.off_T);
    w.Tin = h->at<double>(L.off_Tin);
    w.U = h->at<double>(L.off_U);
    w.W = h->at<double>(L.off_W);
    w.ts_tiles = h->at<double>(L.off_ts_tiles);
    w.ts_X = h->at<double>(L.off_ts_X);
    w.ts_tau = h->at<double>(L.off_ts_tau);
    w.tree = L.tree;
    w.max_chunks = qr_max_chunks();
    w.split_wgs = h->tuning.qr_split_wgs;
    w.panel = h->tuning.qr_panel;
    w.cq_S = h->at<double>(L.off_cq_S);
    w.cq_ld = L.lda;
    w.cq_part = h->at<double>(L.off_cq_part);
    w.cq_G = h->at<double>(L.off_cq_G);
    w.cq_R = h->at<double>(L.off_cq_R);
    w.status = h->status();
    double *rhs = h->at<double>(L.off_rhs);
    if (!L.mixed) {
        h->mark(4, false);
        GAP_TRY(dev(launch_geqrf(w, s, (use_lookahead(h) && h->la.join) ? &h->la : nullptr)));
        h->mark(4, true);
        const double *qtb = A + L.M * L.lda;
        h->mark(5, false);
        hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((L.M + 255) / 256)), dim3(256), 0, s, qtb, rhs, L.M);
        GAP_TRY(dev(launch_trsv_upper(A, L.lda, L.M, rhs, c_out, h->tsync(), s)));
        h->mark(5, true);
        GAP_TRY(dev(launch_sumsq(qtb + L.M, L.N, h->misc(), h->misc() + 1, h->counters() + 8, s)));
        h->mark(8, false);
        GAP_TRY(dev(launch_diag_fp64(h->diag(nullptr), A, qtb, c_out, h->diag_out(), s)));
        h->mark(8, true);
    } else {
        // FP32 copy of [A | b], FP32 Householder QR (FP64 reflector norms), then
        // FP64 refinement against the untouched FP64 [A | b]
        float *A32 = h->at<float>(L.off_A32);
        w.A32 = A32;
        w.W32 = h->at<float>(L.off_W32);
        h->mark(4, false);
        if (L.lp) {
            // rows 0..N-1 came from the low-precision K_NM; L^T and b come from the FP64 [A | b]
            GAP_TRY(dev(launch_convert_block_f64_f32(A, A32, L.lda, L.N, L.lda, 0, L.M, s)));
            GAP_TRY(dev(launch_convert_block_f64_f32(A, A32, L.lda, 0, L.lda, L.M, L.M + 1, s)));
        } else {
            GAP_TRY(dev(launch_convert_f64_f32(A, A32, L.lda * L.ncols, s)));
        }
        GAP_TRY(dev(launch_geqrf(w, s, (use_lookahead(h) && h->la.join) ? &h->la : nullptr)));
        h->mark(4, true);
        h->mark(5, false);
        GAP_TRY(dev(launch_copy_f32_f64(A32 + L.M * L.lda, rhs, L.M, s)));
        GAP_TRY(dev(launch_trsv_upper_f32(A32, L.lda, L.M, rhs, c_out, h->tsync(), nullptr, s)));
        h->mark(5, true);
        RefineWork rw{};
        rw.A = A;
        rw.lda = L.lda;
        rw.m = L.m;
        rw.n = L.M;
        rw.R32 = A32;
        rw.c = c_out;
        rw.r = h->at<double>(L.off_r);
        rw.s = h->at<double>(L.off_s);
        rw.z = h->at<double>(L.off_z);
        rw.dc = h->at<double>(L.off_dc);
        rw.p = h->at<double>(L.off_p);
        rw.q = h->at<double>(L.off_q);
        rw.part = h->at<double>(L.off_part);
        rw.rnorm_part = h->at<double>(L.off_rnorm);
        rw.done = h->at<int32_t>(L.off_flags);
        rw.iters = h->at<int32_t>(L.off_flags) + 1;
        rw.mode = h->at<int32_t>(L.off_flags) + 3;
        rw.stats = h->at<double>(L.off_stats);
        rw.tol = h->p.refine_tol;
        rw.status = h->status();
        rw.sync = h->tsync();
        h->mark(6, false);
        GAP_TRY(dev(launch_refine(rw, h->p.max_refine_iters, s)));
        h->mark(6, true);
        GAP_TRY(dev(launch_check_finite(c_out, L.M, h->status(), s)));
        hipLaunchKernelGGL(copy_kernel, dim3(1), dim3(256), 0, s, rw.stats, h->misc(), (int64_t)1);
        // the refinement's last pass left A^T r at the returned c in rw.s
        h->mark(8, false);
        GAP_TRY(dev(launch_diag_mixed(h->diag(rw.s), A32, A + L.M * L.lda, L.m, rw.stats, c_out, h->diag_out(), s)));
        h->mark(8, true);
    }
    h->state = ST_SOLVED;
    if (info)
        return gap_sync(h, info);
    return GAP_OK;
}

gap_status gap_predict(gap_handle h, const double *x_atoms, int64_t n_atoms, const int64_t *offsets,
                       int64_t n_configs, const double *c, double *y_out)
{
    if (!h || !x_atoms || !offsets || !c || !y_out || n_atoms < 0 || n_configs < 1)
        return GAP_EINVAL;
    if ((h->state < ST_BUILT && !h->model_only) || !h->x_sparse)
        return GAP_ESTATE;
    const double sw2 = h->p.sigma_w * h->p.sigma_w;
    const int64_t M = h->model_only ? h->model_M : h->L.M;
    return dev(launch_predict(x_atoms, n_atoms, offsets, n_configs, h->x_sparse, M, h->p.d, h->p.zeta, sw2, c,
                              y_out, predict_status(h), h->stream));
}

gap_status gap_set_model(gap_handle h, const double *x_sparse, int64_t M)
{
    if (!h || !x_sparse || M < 1)
        return GAP_EINVAL;
    if (!h->model_only) {
        // the handle becomes predict-only: a fit's workspace is no longer used
        h->ws = nullptr;
        h->ws_bytes = 0;
        h->L = Layout();
        h->state = ST_CREATED;
    }
    h->x_sparse = x_sparse;
    h->model_M = M;
    h->model_only = true;
    return GAP_OK;
}

gap_status gap_set_stream(gap_handle h, void *stream)
{
    if (!h)
        return GAP_EINVAL;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    return GAP_OK;
}

gap_status gap_layout(gap_handle h, gap_layout_info *out)
{
    if (!h || !out)
        return GAP_EINVAL;
    if (h->state < ST_BUILT)
        return GAP_ESTATE;
    out->A_aug = h->A();
    out->lda = h->L.lda;
    out->ncols = h->L.ncols;
    out->N = h->L.N;
    out->M = h->L.M;
    out->n_atoms = h->L.n_atoms;
    out->tau = h->at<double>(h->L.off_tau);
    out->device_status = h->status();
    out->A32 = h->L.mixed ? h->at<float>(h->L.off_A32) : nullptr;
    return GAP_OK;
}

gap_status gap_stage_times(gap_handle h, float *ms, int n)
{
    if (!h || !ms || n < 0)
        return GAP_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess)
        return GAP_EDEVICE;
    for (int i = 0; i < n && i < N_STAGES; ++i) {
        ms[i] = 0.0f;
        if (h->timing && h->timed[i]) {
            float v = 0.0f;
            if (hipEventElapsedTime(&v, h->ev[2 * i], h->ev[2 * i + 1]) == hipSuccess)
                ms[i] = v;
        }
    }
    return GAP_OK;
}

gap_status gap_set_tuning(gap_handle h, const gap_tuning *t)
{
    if (!h || !t)
        return GAP_EINVAL;
    if (t->qr_split_wgs != 0 && (t->qr_split_wgs < 256 || t->qr_split_wgs > 65536))
        return GAP_EINVAL;
    if (t->qr_panel != 0 && t->qr_panel != 1)
        return GAP_EINVAL;
    if (t->qr_lookahead < 0 || t->qr_lookahead > 2)
        return GAP_EINVAL;
    if (t->qr_free_cus < 0 || t->qr_free_cus > 128)
        return GAP_EINVAL;
    if (t->knm_bn != 0 && t->knm_bn != 32 && t->knm_bn != 64)
        return GAP_EINVAL;
    h->tuning = *t;
    return GAP_OK;
}

gap_status gap_destroy(gap_handle h)
{
    if (!h)
        return GAP_EINVAL;
    destroy_handle(h);
    return GAP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free fit.  Its scratch is this file-scope device array: each GPU
// the library runs on holds its own copy until the process ends.  Host code
// never uses the array's name as an address; it takes the device address
// from hipGetSymbolAddress, once per device, with that device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[GAP_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[MAX_DEVICES] = {};

// This device's copy of `scratch` (looked up on its first use).
gap_status static_scratch(int device, char **out)
{
    if (device < 0 || device >= MAX_DEVICES)
        return GAP_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return GAP_EDEVICE;
        g_scratch_ptr[device] = static_cast<char *>(ptr);
    }
    *out = g_scratch_ptr[device];
    return GAP_OK;
}

}  // namespace

extern "C" {

size_t gap_static_scratch_bytes(void) { return GAP_STATIC_SCRATCH_BYTES; }

gap_status gap_fit_static(const gap_params *p, void *stream, const double *x_atoms, int64_t n_atoms,
                          const int64_t *config_offsets, int64_t n_configs, const double *x_sparse, int64_t M,
                          const double *sigma, const double *y, double *c_out, gap_solve_info *info)
{
    if (!valid_params(p) || (p->flags & GAP_FLAG_TIMING))
        return GAP_EINVAL;
    if (!x_atoms || !config_offsets || !x_sparse || !sigma || !y || !c_out || n_atoms < 1 || n_configs < 1 ||
        M < 1 || n_configs > INT32_MAX - 1)
        return GAP_EINVAL;
    const size_t need = make_layout(n_configs, n_atoms, M, p->precision, p->d, p->flags).total;
    if (need > GAP_STATIC_SCRATCH_BYTES)
        return GAP_ENOMEM;
    gap_handle_s h;  // on the stack: no timing events, no look-ahead stream
    h.p = *p;
    h.stream = reinterpret_cast<hipStream_t>(stream);
    if (hipGetDevice(&h.device) != hipSuccess)
        return GAP_EDEVICE;
    char *base = nullptr;
    GAP_TRY(static_scratch(h.device, &base));
    h.ws = base;
    h.ws_bytes = GAP_STATIC_SCRATCH_BYTES;
    h.state = ST_BOUND;
    h.tuning.qr_lookahead = 1;  // the whole QR on `stream`
    GAP_TRY(gap_build_knm(&h, x_atoms, n_atoms, config_offsets, n_configs, x_sparse, M, sigma));
    return gap_solve(&h, y, c_out, info);
}

}  // extern "C"
