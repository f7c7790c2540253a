// ibsn_api.hip -- the C ABI of libibsn.so (include/ibsn.h): context and workspace
// management, argument checks, the pass-level entry points and the IBSN solver loop
// (Algorithm 2 with the practical stop schedule of Section 5).
//
// The host only sequences kernels and reads back the scalars a decision needs
// (||g||, the Armijo decrease, D_phi and the certificate, the CG done flag).  All
// arithmetic on problem data runs in the kernels of dense_*.hip, sparse_ops.hip
// and solver_kernels.hip.
#include "../../include/ibsn.h"
#include "ibsn_internal.h"
#include "solver_kernels.h"

#include <algorithm>
#include <atomic>
#include <numeric>
#include <mutex>
#include <thread>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace ibsn;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct ibsn_csr {
    ibsn_ctx *ctx = nullptr;
    int64_t m = 0, n = 0;
    int64_t nnz = 0;       // host copy (valid after sparsify)
    int64_t istar = -1;    // host copy
    int64_t m2 = 0;        // host copy: sum over rows != istar of len^2 (entries of P'^T A P')
    int f32 = 0;           // values stored as FP32 (mixed-precision sparsify)
    DevBuf col, val, len, colptr, colcnt, rowidx, cval, mask, off, d, istar_dev, nnz_dev;
};

// Device memory of ibsn_hvp_noalloc, for callers that cannot allocate: u = a o (P_rho v)
// (up to IBSN_NOALLOC_MAX_M rows) followed by the dense row's CG_MAX_STAR chunk partials.
// Each device holds its own copy until the process ends.  Host code never uses the array's
// name as an address: ibsn_create looks up each device's copy once (scratch_dev).
static __device__ __align__(256) double scratch[IBSN_NOALLOC_MAX_M + CG_MAX_STAR];
static double *scratch_dev[64];
static std::mutex scratch_mu;

struct ibsn_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    double *scratch = nullptr;   // this device's copy of `scratch` (device address)
    int num_cus = 256;
    size_t max_lds = 65536;
    std::string err;
    // workspace
    DevBuf w, wlo, lcv, clpart, colpart, colpart2, rowpart, rowpart2, scal, colv, cvec, gvec, yv, ecv, psiv, zv;
    DevBuf erv, zgv;
    DevBuf stopout, tauv, cg_x, cg_r, cg_r2, cg_p, cg_Ap, cg_au, cg_star, cg_pap, cg_rr, cg_scal;
    DevBuf cg_pp;                  // partial sums and barrier state of the one-launch CG
    DevBuf cg_mcnt, cg_mptr, cg_mcol, cg_mval, cg_w;   // M = P'^T diag(a) P' and w (2 n)
    int cg_mode = 0;               // IBSN_CG_AUTO / _LAUNCHES / _PERSISTENT / _SINGLE
    bool coop_off = false;         // no cooperative launches (several contexts at once)
    int64_t split_cols = 0;        // rows wider than this are split (0: wider than a tile)
    int csc_fill = IBSN_CSC_AUTO;  // fill of the transpose (ibsn_set_csc_fill)
    DevBuf wd_M, wd_S, wd_f, wd_rr, wd_len;   // per-block row arrays of split rows
    struct Tuned {                 // plans chosen by ibsn_autotune, per problem shape
        int64_t m, n;
        int kind, mixed;
        RowPlan rp;
    };
    std::vector<Tuned> tuned;
    int cg_blocks = 0;             // grid of the one-launch CG (0: from the problem size)
    bool coop = false;             // the device supports cooperative launches
    double *host_scal = nullptr;   // pinned, SC_NSLOT + 16
    double *cg_host = nullptr;     // pinned, 2 * CG_NSLOT: CG state records, double-buffered
    hipEvent_t cg_ev[2] = {nullptr, nullptr};
    ibsn_csr *solver_csr = nullptr;
    std::vector<ibsn_csr *> csrs;  // handles returned by ibsn_sparsify and not yet freed
    // solver state (grow-only, reused across ibsn_solve calls)
    DevBuf sv_r, sv_s, sv_g, sv_M, sv_S, sv_Mt, sv_St, sv_ct, sv_gt, sv_D, sv_c, sv_gv;
    // kernel timing (HIP events around the main kernel of each phase)
    bool timing = false;
    double kt_ms[IBSN_KT_N] = {0};
    int64_t kt_count[IBSN_KT_N] = {0};
    std::vector<hipEvent_t> ev_free;
    struct Pending {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
};

namespace {

int fail(ibsn_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

#define CKH(call)                                                                           \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, IBSN_ERR_HIP, "%s failed: %s (%s:%d)", #call,                  \
                        hipGetErrorString(e_), __FILE__, __LINE__);                          \
    } while (0)

#define CKI(call)                 \
    do {                          \
        int r_ = (call);          \
        if (r_ < 0)               \
            return r_;            \
    } while (0)

int ensure(ibsn_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes == 0)
        bytes = 16;
    if (b.bytes >= bytes)
        return IBSN_OK;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        if (e != hipSuccess)
            return fail(ctx, IBSN_ERR_HIP, "hipFree: %s", hipGetErrorString(e));
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, IBSN_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    b.bytes = bytes;
    return IBSN_OK;
}

void release(DevBuf &b)
{
    if (b.p)
        (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

template <typename T>
T *P(DevBuf &b)
{
    return reinterpret_cast<T *>(b.p);
}

// Width of the column blocks of a split row, or 0 when rows are not split.  Rows are split
// when they exceed the register tiles (10240 columns for an FP64 or points cost, 20000 for
// an FP32 cost) or the width set by ibsn_set_row_split; blocks are then at most 10240
// columns (FP64, points), 12288 (FP32, so that the low parts of w still fit) or the set
// width, of equal width rounded up to a multiple of 64 except the last.
int64_t split_width(const ibsn_ctx *ctx, const ibsn_problem *p)
{
    const int64_t n = p->n;
    const int64_t narrow = p->cost_kind == IBSN_COST_F32 ? IBSN_MAX_N_F32 : IBSN_MAX_N_F64;
    const int64_t lim = ctx->split_cols > 0 ? ctx->split_cols : narrow;
    if (n <= lim)
        return 0;
    const int64_t blk = ctx->split_cols > 0 ? ctx->split_cols
                        : (p->cost_kind == IBSN_COST_F32 ? (int64_t)LO_MAX_COLS
                                                         : (int64_t)IBSN_MAX_N_F64);
    const int64_t nb = (n + blk - 1) / blk;
    const int64_t bw = ((n + nb - 1) / nb + 63) / 64 * 64;
    return bw < blk ? bw : blk;
}

int check_problem(ibsn_ctx *ctx, const ibsn_problem *p)
{
    if (!ctx)
        return IBSN_ERR_INVALID_ARG;
    if (!p)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "problem is NULL");
    if (p->m < 1 || p->n < 1)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "m=%lld, n=%lld: both must be >= 1",
                    (long long)p->m, (long long)p->n);
    if (p->m > 0x7fffffffLL || p->n > 0x7fffffffLL || p->m * p->n > (int64_t)1 << 40)
        return fail(ctx, IBSN_ERR_UNSUPPORTED, "m*n too large");
    if (!(p->eta > 0.0) || !std::isfinite(p->eta))
        return fail(ctx, IBSN_ERR_INVALID_ARG, "eta=%g must be finite and > 0", p->eta);
    if (p->cost_kind != IBSN_COST_F64 && p->cost_kind != IBSN_COST_F32 &&
        p->cost_kind != IBSN_COST_POINTS)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "cost_kind=%d unknown", p->cost_kind);
    if (p->precision != IBSN_PREC_F64 && p->precision != IBSN_PREC_MIXED)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "precision=%d unknown", p->precision);
    if (p->cost_kind == IBSN_COST_POINTS) {
        if (!p->C || !p->y || !p->a || !p->b)
            return fail(ctx, IBSN_ERR_INVALID_ARG, "points cost needs device x (C), y, a and b");
        if (p->ldc != 2 && p->ldc != 3)
            return fail(ctx, IBSN_ERR_UNSUPPORTED, "points of dimension %lld (2 or 3 supported)",
                        (long long)p->ldc);
        if (!(p->cost_scale > 0.0) || !std::isfinite(p->cost_scale))
            return fail(ctx, IBSN_ERR_INVALID_ARG, "cost_scale=%g must be finite and > 0",
                        p->cost_scale);
        if (((uintptr_t)p->C % 8) != 0 || ((uintptr_t)p->y % 8) != 0)
            return fail(ctx, IBSN_ERR_INVALID_ARG, "x and y must be 8-byte aligned");
        const int64_t wp = split_width(ctx, p) ? split_width(ctx, p) : p->n;
        if ((size_t)wp * sizeof(double) + 3584 > ctx->max_lds)
            return fail(ctx, IBSN_ERR_UNSUPPORTED, "n=%lld needs %zu bytes of LDS (device max %zu)",
                        (long long)wp, (size_t)wp * 8 + 3584, ctx->max_lds);
        return IBSN_OK;
    }
    if (!p->C || !p->a || !p->b)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "C, a and b must be device pointers");
    if (p->ldc < p->n)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "ldc=%lld < n=%lld", (long long)p->ldc,
                    (long long)p->n);
    // rows wider than the register tiles are split into column blocks (split_width)
    const int64_t wmax = split_width(ctx, p) ? split_width(ctx, p) : p->n;
    const size_t es = p->cost_kind == IBSN_COST_F64 ? 8 : 4;
    if (((uintptr_t)p->C % es) != 0)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "C must be aligned to its element size");
    // the row passes stage an n-vector in LDS beside at most 3.5 KB of their own (each
    // launch also checks its exact total against the device limit)
    if ((size_t)wmax * sizeof(double) + 3584 > ctx->max_lds)
        return fail(ctx, IBSN_ERR_UNSUPPORTED, "n=%lld needs %zu bytes of LDS (device max %zu)",
                    (long long)wmax, (size_t)wmax * 8 + 3584, ctx->max_lds);
    return IBSN_OK;
}

int check_center(ibsn_ctx *ctx, const ibsn_center *c)
{
    if (!c || !c->s)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "center (k, r, s) with device s is required");
    if (c->k < 0)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "center k=%lld < 0", (long long)c->k);
    int e = 0;
    if (!(c->quantum >= DBL_MIN) || !std::isfinite(c->quantum) ||
        std::frexp(c->quantum, &e) != 0.5)
        return fail(ctx, IBSN_ERR_INVALID_ARG,
                    "center quantum=%g must be a normal power of two", c->quantum);
    return IBSN_OK;
}

// grid spacing 2^(e-50) for a bound 2^(e-1) <= B < 2^e (see ibsn_center)
double quantum_of(double B)
{
    if (!(B >= 1.0))
        B = 1.0;
    return std::ldexp(1.0, std::ilogb(B) + 1 - 50);
}

int plan_for(ibsn_ctx *ctx, const ibsn_problem *p, RowPlan *rp)
{
    if (const int64_t bw = split_width(ctx, p)) {
        if (!plan_rows(p->m, bw, p->cost_kind, ctx->num_cus, rp))
            return fail(ctx, IBSN_ERR_UNSUPPORTED, "no row tile for blocks of %lld columns",
                        (long long)bw);
        rp->bw = bw;
        rp->nb = (int)((p->n + bw - 1) / bw);
        return IBSN_OK;
    }
    if (!plan_rows(p->m, p->n, p->cost_kind, ctx->num_cus, rp))
        return fail(ctx, IBSN_ERR_UNSUPPORTED, "no row tile for n=%lld", (long long)p->n);
    const int mixed = p->precision == IBSN_PREC_MIXED ? 1 : 0;
    for (const auto &t : ctx->tuned)
        if (t.m == p->m && t.n == p->n && t.kind == p->cost_kind && t.mixed == mixed) {
            *rp = t.rp;
            break;
        }
    return IBSN_OK;
}

// per-call workspace sized for (m, n, grid)
int ensure_ws(ibsn_ctx *ctx, const ibsn_problem *p, const RowPlan &rp)
{
    const size_t n = (size_t)p->n, m = (size_t)p->m, G = (size_t)rp.grid * (size_t)rp.nb;
    if (rp.nb > 1) {
        const size_t nb = (size_t)rp.nb;
        CKI(ensure(ctx, ctx->wd_M, nb * m * 8));
        CKI(ensure(ctx, ctx->wd_S, nb * m * 8));
        CKI(ensure(ctx, ctx->wd_f, m * 8));
        CKI(ensure(ctx, ctx->wd_rr, 4 * nb * m * 8));
        CKI(ensure(ctx, ctx->wd_len, nb * m * 4));
    }
    CKI(ensure(ctx, ctx->w, n * 8));
    CKI(ensure(ctx, ctx->wlo, n * 8));
    CKI(ensure(ctx, ctx->lcv, n * 8));
    CKI(ensure(ctx, ctx->clpart, 2 * (size_t)COLLSE_MAX_RB * n * 8));
    CKI(ensure(ctx, ctx->colpart, G * n * 8));
    CKI(ensure(ctx, ctx->colpart2, G * n * 8));
    CKI(ensure(ctx, ctx->rowpart, G * STOP2_NSLOT * 8));
    CKI(ensure(ctx, ctx->rowpart2, G * 8));
    CKI(ensure(ctx, ctx->scal, SC_NSLOT * 8));
    CKI(ensure(ctx, ctx->colv, n * 8));
    CKI(ensure(ctx, ctx->cvec, n * 8));
    CKI(ensure(ctx, ctx->gvec, n * 8));
    CKI(ensure(ctx, ctx->yv, n * 8));
    CKI(ensure(ctx, ctx->ecv, n * 8));
    CKI(ensure(ctx, ctx->psiv, n * 8));
    CKI(ensure(ctx, ctx->zv, m * 8));
    CKI(ensure(ctx, ctx->erv, m * 8));
    CKI(ensure(ctx, ctx->zgv, m * 8));
    CKI(ensure(ctx, ctx->stopout, 16 * 8));
    CKI(ensure(ctx, ctx->tauv, n * 8));
    return IBSN_OK;
}

DenseArgs dense_args(ibsn_ctx *ctx, const ibsn_problem *p, int64_t k, double q, int mixed = 0)
{
    DenseArgs d;
    d.mixed = mixed;
    d.q = q;
    d.C = p->C;
    d.ldc = p->ldc;
    d.m = p->m;
    d.n = p->n;
    d.cost_kind = p->cost_kind;
    d.py = p->cost_kind == IBSN_COST_POINTS ? p->y : nullptr;
    d.pscale = p->cost_kind == IBSN_COST_POINTS ? p->cost_scale : 0.0;
    d.pdim = p->cost_kind == IBSN_COST_POINTS ? (int)p->ldc : 0;
    d.sigma = (double)(k + 1) / p->eta;
    d.w = P<double>(ctx->w);
    d.wlo = P<double>(ctx->wlo);
    d.a = p->a;
    d.ldo = p->n;
    d.coff = 0;
    return d;
}

// whether the dense passes of this problem carry the low parts of the potentials: every
// tile except the FP32-cost ones wider than LO_MAX_COLS columns (the block width of a
// split row)
int lo_split(const ibsn_ctx *ctx, const ibsn_problem *p)
{
    const int64_t bw = split_width(ctx, p);
    return (p->cost_kind != IBSN_COST_F32 || (bw ? bw : p->n) <= LO_MAX_COLS) ? 1 : 0;
}

int read_scal(ibsn_ctx *ctx, int count = SC_NSLOT)
{
    CKH(hipMemcpyAsync(ctx->host_scal, ctx->scal.p, sizeof(double) * count, hipMemcpyDeviceToHost,
                       ctx->stream));
    CKH(hipStreamSynchronize(ctx->stream));
    return IBSN_OK;
}

// kernel timing: tic() records a start event, toc() an end event for phase `kind`
hipEvent_t take_event(ibsn_ctx *ctx)
{
    if (!ctx->ev_free.empty()) {
        hipEvent_t e = ctx->ev_free.back();
        ctx->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

void drain_events(ibsn_ctx *ctx)
{
    if (ctx->pending.empty())
        return;
    (void)hipEventSynchronize(ctx->pending.back().b);
    for (auto &p : ctx->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            ctx->kt_ms[p.kind] += ms;
            ctx->kt_count[p.kind] += 1;
        }
        ctx->ev_free.push_back(p.a);
        ctx->ev_free.push_back(p.b);
    }
    ctx->pending.clear();
}

struct KTimer {
    ibsn_ctx *ctx;
    int kind;
    hipEvent_t a = nullptr;
    KTimer(ibsn_ctx *c, int k) : ctx(c), kind(k)
    {
        if (ctx->timing) {
            a = take_event(ctx);
            if (a)
                (void)hipEventRecord(a, ctx->stream);
        }
    }
    ~KTimer()
    {
        if (ctx->timing && a) {
            hipEvent_t b = take_event(ctx);
            if (b) {
                (void)hipEventRecord(b, ctx->stream);
                ctx->pending.push_back({kind, a, b});
                if (ctx->pending.size() >= 512)
                    drain_events(ctx);
            } else {
                ctx->ev_free.push_back(a);
            }
        }
    }
};

// ---------------------------------------------------------------------------------
// pass-level building blocks (also used by the solver)
// ---------------------------------------------------------------------------------
// Column block b of a split row: columns [j0, j0 + w), its tile plan (the last block's own
// tile, on the same grid) and its pass arguments (cost, y, w and its low parts from column
// j0; the m x n outputs keep the row pitch n).
struct Block {
    int64_t j0, w;
    RowPlan rp;
    DenseArgs d;
};
Block block_of(const ibsn_ctx *ctx, const RowPlan &rp, const DenseArgs &d, int b)
{
    Block k;
    k.j0 = (int64_t)b * rp.bw;
    k.w = std::min<int64_t>(rp.bw, d.n - k.j0);
    k.rp = rp;
    if (k.w != rp.bw) {
        plan_rows(d.m, k.w, d.cost_kind, ctx->num_cus, &k.rp);
        k.rp.grid = rp.grid;
    }
    k.d = d;
    k.d.n = k.w;
    k.d.ldo = d.n;
    k.d.coff = k.j0;
    if (d.cost_kind == IBSN_COST_POINTS)
        k.d.py = d.py + k.j0 * d.pdim;
    else
        k.d.C = (const char *)d.C + k.j0 * (d.cost_kind == IBSN_COST_F32 ? 4 : 8);
    k.d.w = d.w + k.j0;
    k.d.wlo = d.wlo + k.j0;
    return k;
}

// eval at the current ctx->w (already formed); writes M, S, lse, c, g, plan; objective to
// scal[SC_OBJ] when r != null (needs gamma for b^T gamma); norms of g to scal.
int run_eval(ibsn_ctx *ctx, const ibsn_problem *p, const RowPlan &rp, int64_t k, double q,
             const double *r, const double *gamma, double *M, double *S, double *lse, double *c,
             double *g, double *plan, int mixed)
{
    hipStream_t st = ctx->stream;
    DenseArgs d = dense_args(ctx, p, k, q, mixed);
    if (rp.nb > 1) {
        // each block's (M, S), the rows joined, then each block's column partials from the
        // whole row's shift and a_i / S_i
        KTimer kt(ctx, mixed ? IBSN_KT_EVAL_MIXED : IBSN_KT_EVAL);
        const int64_t m = p->m;
        double *Mb = P<double>(ctx->wd_M), *Sb = P<double>(ctx->wd_S), *f = P<double>(ctx->wd_f);
        for (int b = 0; b < rp.nb; ++b) {
            const Block bk = block_of(ctx, rp, d, b);
            CKH(launch_eval(bk.rp, bk.d, nullptr, Mb + b * m, Sb + b * m, nullptr, nullptr,
                            nullptr, nullptr, st));
        }
        CKH(launch_wide_eval_rows(m, rp.nb, Mb, Sb, p->a, r, M, S, lse, f,
                                  P<double>(ctx->rowpart), rp.grid, st));
        for (int b = 0; b < rp.nb; ++b) {
            const Block bk = block_of(ctx, rp, d, b);
            CKH(launch_eval(bk.rp, bk.d, nullptr, nullptr, nullptr, nullptr,
                            plan ? plan + bk.j0 : nullptr, P<double>(ctx->colpart), nullptr, st,
                            M, f));
            CKH(launch_colreduce(P<double>(ctx->colpart), rp.grid, bk.w, c + bk.j0,
                                 p->b + bk.j0, g + bk.j0, st));
        }
    } else {
        {
            KTimer kt(ctx, mixed ? IBSN_KT_EVAL_MIXED : IBSN_KT_EVAL);
            CKH(launch_eval(rp, d, r, M, S, lse, plan, P<double>(ctx->colpart),
                            P<double>(ctx->rowpart), st));
        }
        KTimer kt(ctx, IBSN_KT_COLRED);
        CKH(launch_colreduce(P<double>(ctx->colpart), rp.grid, p->n, c, p->b, g, st));
    }
    CKH(sk_gnorms(p->n, g, P<double>(ctx->scal), st));
    if (r && gamma) {
        CKH(sk_dot_slot(p->n, p->b, gamma, SC_BG, P<double>(ctx->scal), st));
        CKH(sk_sum_parts(rp.grid, 1, 0, P<double>(ctx->rowpart), p->eta, -1.0, SC_BG, SC_OBJ, 0,
                         P<double>(ctx->scal), st));
    }
    return IBSN_OK;
}

// trial at the grid point w + grid(t Delta/eta) (step kept in ctx->tauv): writes Mn, Sn,
// cn, gn; scal[SC_DL] = dL.
int run_trial(ibsn_ctx *ctx, const ibsn_problem *p, const RowPlan &rp, int64_t k, double q,
              const double *M, const double *Delta, double t, double *Mn, double *Sn, double *cn,
              double *gn, int mixed)
{
    hipStream_t st = ctx->stream;
    DenseArgs d = dense_args(ctx, p, k, q, mixed);
    double *scal = P<double>(ctx->scal);
    CKH(sk_trial_prep(p->n, t, p->eta, q, lo_split(ctx, p), Delta, p->b, P<double>(ctx->tauv), P<double>(ctx->colv),
                      scal, st));
    if (rp.nb > 1) {
        // each block's row sums, the rows joined (decrease, new state, a_i / Z_i), then each
        // block's column partials
        KTimer kt(ctx, mixed ? IBSN_KT_TRIAL_MIXED : IBSN_KT_TRIAL);
        const int64_t m = p->m;
        double *rr = P<double>(ctx->wd_rr), *f = P<double>(ctx->wd_f);
        for (int b = 0; b < rp.nb; ++b) {
            const Block bk = block_of(ctx, rp, d, b);
            CKH(launch_trial(bk.rp, bk.d, M, P<double>(ctx->colv) + bk.j0, scal, nullptr, nullptr,
                             nullptr, nullptr, st, rr + 4 * m * b, nullptr));
        }
        CKH(launch_wide_trial_rows(m, rp.nb, rr, p->a, M, scal, q, Mn, Sn, f,
                                   P<double>(ctx->rowpart), rp.grid, st));
        for (int b = 0; b < rp.nb; ++b) {
            const Block bk = block_of(ctx, rp, d, b);
            CKH(launch_trial(bk.rp, bk.d, M, P<double>(ctx->colv) + bk.j0, scal, nullptr, nullptr,
                             P<double>(ctx->colpart), nullptr, st, nullptr, f));
            CKH(launch_colreduce(P<double>(ctx->colpart), rp.grid, bk.w, cn + bk.j0,
                                 p->b + bk.j0, gn + bk.j0, st));
        }
    } else {
        {
            KTimer kt(ctx, mixed ? IBSN_KT_TRIAL_MIXED : IBSN_KT_TRIAL);
            CKH(launch_trial(rp, d, M, P<double>(ctx->colv), scal, Mn, Sn, P<double>(ctx->colpart),
                             P<double>(ctx->rowpart), st));
        }
        KTimer kt(ctx, IBSN_KT_COLRED);
        CKH(launch_colreduce(P<double>(ctx->colpart), rp.grid, p->n, cn, p->b, gn, st));
    }
    CKH(sk_gnorms(p->n, gn, scal, st));
    // dL = eta * sum_i a_i delta_i - eta * b^T tau
    CKH(sk_sum_parts(rp.grid, 1, 0, P<double>(ctx->rowpart), p->eta, -p->eta, SC_TB, SC_DL, 0,
                     scal, st));
    return IBSN_OK;
}

// stop test + certificate at the state (w, M, S); out (device, 10 doubles).
// c_state: the state's column sums c = X^T 1 when the caller holds them (the solver does).
// X = diag(a) P with P row-stochastic, so X 1 = a and Algorithm 3's first scaling is
// z = min(a / X1, 1) = 1, F = X: pass 1 (which forms z and the column sums of X and F)
// is then skipped, z is 1 and both column sums are c_state.  Without c_state pass 1 runs
// as Algorithm 3 states it.
int run_stop(ibsn_ctx *ctx, const ibsn_problem *p, const RowPlan &rp, int64_t k, double q,
             const double *gamma, const double *M, const double *S, double *xhat,
             const double *c_state = nullptr)
{
    hipStream_t st = ctx->stream;
    DenseArgs d = dense_args(ctx, p, k, q);
    double *scal = P<double>(ctx->scal);
    const double *colX = P<double>(ctx->cvec);   // column sums of X
    const double *colF = P<double>(ctx->colv);   // column sums of F = diag(z) X
    int rowres_parts = rp.grid;                  // partials of sum_i (X1 - a)_i^2
    const int64_t m = p->m;
    double *rr = P<double>(ctx->wd_rr);
    if (c_state) {
        CKH(sk_fill(p->m, 1.0, P<double>(ctx->zv), st));
        colX = colF = c_state;
        rowres_parts = 0;   // X1 = a
    } else if (rp.nb > 1) {
        // the blocks' row sums of X (and column sums of X), z from the joined rows, then the
        // column sums of z X
        KTimer kt(ctx, IBSN_KT_STOP1);
        for (int b = 0; b < rp.nb; ++b) {
            const Block bk = block_of(ctx, rp, d, b);
            CKH(launch_stop1(bk.rp, bk.d, M, S, nullptr, P<double>(ctx->colpart), nullptr, nullptr,
                             st, rr + b * m, nullptr));
            CKH(launch_colreduce(P<double>(ctx->colpart), rp.grid, bk.w,
                                 P<double>(ctx->cvec) + bk.j0, nullptr, nullptr, st));
        }
        CKH(launch_wide_stop1_rows(m, rp.nb, rr, p->a, P<double>(ctx->zv),
                                   P<double>(ctx->rowpart2), rp.grid, st));
        for (int b = 0; b < rp.nb; ++b) {
            const Block bk = block_of(ctx, rp, d, b);
            CKH(launch_stop1(bk.rp, bk.d, M, S, nullptr, nullptr, P<double>(ctx->colpart2), nullptr,
                             st, nullptr, P<double>(ctx->zv)));
            CKH(launch_colreduce(P<double>(ctx->colpart2), rp.grid, bk.w,
                                 P<double>(ctx->colv) + bk.j0, nullptr, nullptr, st));
        }
    } else {
        {
            KTimer kt(ctx, IBSN_KT_STOP1);
            CKH(launch_stop1(rp, d, M, S, P<double>(ctx->zv), P<double>(ctx->colpart),
                             P<double>(ctx->colpart2), P<double>(ctx->rowpart2), st));
        }
        CKH(launch_colreduce(P<double>(ctx->colpart), rp.grid, p->n, P<double>(ctx->cvec),
                             nullptr, nullptr, st));
        CKH(launch_colreduce(P<double>(ctx->colpart2), rp.grid, p->n, P<double>(ctx->colv),
                             nullptr, nullptr, st));
    }
    CKH(sk_stop_prep(p->n, d.sigma, p->b, d.w, d.wlo, gamma, colX, colF, P<double>(ctx->yv),
                     P<double>(ctx->ecv), P<double>(ctx->psiv), scal, st));
    Stop2Vec v;
    v.gamma = gamma;
    v.psi = P<double>(ctx->psiv);
    v.y = P<double>(ctx->yv);
    v.ec = P<double>(ctx->ecv);
    v.z = P<double>(ctx->zv);
    v.er_row = P<double>(ctx->erv);
    v.zg_row = P<double>(ctx->zgv);
    v.er1 = scal + SC_ER1;   // read on the device: no host round trip
    int parts = rp.grid;
    if (rp.nb > 1) {
        // pass 2a per block into per-row partials, the rows joined (e_r, zg and the dual
        // sums over all nb * grid slots), then pass 2b per block into its own slots
        KTimer kt(ctx, IBSN_KT_STOP2);
        parts = rp.grid * rp.nb;
        double *rp2 = P<double>(ctx->rowpart);
        for (int b = 0; b < rp.nb; ++b) {
            const Block bk = block_of(ctx, rp, d, b);
            Stop2Vec vb = v;
            vb.gamma += bk.j0;
            vb.psi += bk.j0;
            vb.y += bk.j0;
            CKH(launch_stop2(bk.rp, bk.d, M, S, vb, nullptr, nullptr, st, 1, rr + 3 * m * b));
        }
        CKH(launch_wide_stop2a_rows(m, rp.nb, rr, p->a, v.z, v.er_row, v.zg_row, rp2, parts, st));
        for (int b = 0; b < rp.nb; ++b) {
            const Block bk = block_of(ctx, rp, d, b);
            Stop2Vec vb = v;
            vb.gamma += bk.j0;
            vb.y += bk.j0;
            vb.ec += bk.j0;
            CKH(launch_stop2(bk.rp, bk.d, M, S, vb, xhat ? xhat + bk.j0 : nullptr,
                             rp2 + (int64_t)b * rp.grid * STOP2_NSLOT, st, 2));
        }
    } else {
        KTimer kt(ctx, IBSN_KT_STOP2);
        CKH(launch_stop2(rp, d, M, S, v, xhat, P<double>(ctx->rowpart), st));
    }
    CKH(sk_stop_final(parts, P<double>(ctx->rowpart), P<double>(ctx->rowpart2), rowres_parts,
                      scal, P<double>(ctx->stopout), st));
    return IBSN_OK;
}

int csr_alloc(ibsn_ctx *ctx, ibsn_csr *c, int64_t m, int64_t n)
{
    const size_t mn = (size_t)m * (size_t)n;
    c->m = m;
    c->n = n;
    CKI(ensure(ctx, c->col, mn * 4));
    CKI(ensure(ctx, c->val, mn * 8));
    CKI(ensure(ctx, c->len, (size_t)m * 4));
    CKI(ensure(ctx, c->colptr, ((size_t)n + 1) * 8));
    CKI(ensure(ctx, c->colcnt, (size_t)n * 8));
    CKI(ensure(ctx, c->rowidx, mn * 4));
    CKI(ensure(ctx, c->cval, mn * 8));
    CKI(ensure(ctx, c->mask, (size_t)csc_row_blocks(m) * n * 4));
    CKI(ensure(ctx, c->off, (size_t)csc_row_blocks(m) * n * 4));
    CKI(ensure(ctx, c->d, (size_t)n * 8));
    CKI(ensure(ctx, c->istar_dev, 16));
    CKI(ensure(ctx, c->nnz_dev, 16));
    return IBSN_OK;
}

void csr_release(ibsn_csr *c)
{
    DevBuf *bufs[] = {&c->col, &c->val, &c->len, &c->colptr, &c->colcnt, &c->rowidx,
                      &c->cval, &c->mask, &c->off, &c->d, &c->istar_dev, &c->nnz_dev};
    for (DevBuf *b : bufs)
        release(*b);
}

CsrView csr_view(const ibsn_csr *c);

// sparsify into c at the state (w formed), rho; istar on device in c->istar_dev
int run_sparsify(ibsn_ctx *ctx, const ibsn_problem *p, const RowPlan &rp, int64_t k, double q,
                 const double *M, const double *S, double rho, ibsn_csr *c, int mixed)
{
    hipStream_t st = ctx->stream;
    DenseArgs d = dense_args(ctx, p, k, q, mixed);
    c->f32 = mixed;
    const bool split = rp.nb > 1;
    if (split) {
        // each block's kept entries at its own offset of the row's slot, then the blocks
        // joined per row; d follows from the transpose below
        KTimer kt(ctx, mixed ? IBSN_KT_SPARSIFY_MIXED : IBSN_KT_SPARSIFY);
        const int64_t m = p->m;
        for (int b = 0; b < rp.nb; ++b) {
            const Block bk = block_of(ctx, rp, d, b);
            CKH(launch_sparsify(bk.rp, bk.d, M, S, rho, P<int>(c->istar_dev), P<int32_t>(c->col),
                                c->val.p, P<int32_t>(ctx->wd_len) + b * m, nullptr, st,
                                P<double>(ctx->wd_rr) + b * m));
        }
        CKH(launch_wide_join(m, p->n, rp.nb, rp.bw, P<int32_t>(ctx->wd_len), P<double>(ctx->wd_rr),
                             p->a, P<int>(c->istar_dev), P<int32_t>(c->col), c->val.p, c->f32,
                             P<int32_t>(c->len), P<double>(ctx->wd_f), st));
    } else {
        {
            KTimer kt(ctx, mixed ? IBSN_KT_SPARSIFY_MIXED : IBSN_KT_SPARSIFY);
            CKH(launch_sparsify(rp, d, M, S, rho, P<int>(c->istar_dev), P<int32_t>(c->col),
                                c->val.p, P<int32_t>(c->len), P<double>(ctx->colpart), st));
        }
        CKH(launch_colreduce(P<double>(ctx->colpart), rp.grid, p->n, P<double>(c->d), nullptr,
                             nullptr, st));
    }
    CscWork cw;
    cw.colptr = P<int64_t>(c->colptr);
    cw.colcnt = P<int64_t>(c->colcnt);
    cw.rowidx = P<int32_t>(c->rowidx);
    cw.cval = c->cval.p;
    cw.mask = P<uint32_t>(c->mask);
    cw.off = P<int32_t>(c->off);
    // lanes per row of the fill from the previous factor's mean row length (64 at first)
    cw.lpc = (c->nnz > 0 && (double)c->nnz / (double)c->m < 96.0) ? 16 : 64;
    cw.fill = ctx->csc_fill;
    {
        KTimer kt(ctx, IBSN_KT_CSC);
        CKH(launch_build_csc(p->m, p->n, P<int32_t>(c->col), c->val.p, c->f32,
                             P<int32_t>(c->len), P<int>(c->istar_dev), cw,
                             P<int64_t>(c->nnz_dev), st));
    }
    if (split)
        CKH(launch_wide_d(csr_view(c), P<double>(ctx->wd_f), P<double>(c->d), st));
    CKH(launch_len_sq(p->m, P<int32_t>(c->len), P<int>(c->istar_dev), P<int64_t>(c->nnz_dev) + 1,
                      st));
    int64_t hv[3];
    CKH(hipMemcpyAsync(hv, c->nnz_dev.p, 8, hipMemcpyDeviceToHost, st));
    CKH(hipMemcpyAsync(hv + 1, c->istar_dev.p, 4, hipMemcpyDeviceToHost, st));
    CKH(hipMemcpyAsync(hv + 2, P<int64_t>(c->nnz_dev) + 1, 8, hipMemcpyDeviceToHost, st));
    CKH(hipStreamSynchronize(st));
    c->nnz = hv[0];
    c->istar = (int64_t)(int32_t)(hv[1] & 0xffffffff);
    c->m2 = hv[2];
    return IBSN_OK;
}

CsrView csr_view(const ibsn_csr *c)
{
    CsrView v;
    v.m = c->m;
    v.n = c->n;
    v.col = (const int32_t *)c->col.p;
    v.val = c->val.p;
    v.f32 = c->f32;
    v.len = (const int32_t *)c->len.p;
    v.istar = (const int *)c->istar_dev.p;
    v.colptr = (const int64_t *)c->colptr.p;
    v.rowidx = (const int32_t *)c->rowidx.p;
    v.cval = c->cval.p;
    v.d = (const double *)c->d.p;
    return v;
}

int ensure_cg(ibsn_ctx *ctx, int64_t m, int64_t n)
{
    CKI(ensure(ctx, ctx->cg_x, n * 8));
    CKI(ensure(ctx, ctx->cg_r, n * 8));
    CKI(ensure(ctx, ctx->cg_r2, n * 8));
    CKI(ensure(ctx, ctx->cg_p, n * 8));
    CKI(ensure(ctx, ctx->cg_Ap, n * 8));
    CKI(ensure(ctx, ctx->cg_au, m * 8));
    CKI(ensure(ctx, ctx->cg_star, CG_MAX_STAR * 8));
    CKI(ensure(ctx, ctx->cg_pap, CG_MAX_COLGROUPS * 8));
    CKI(ensure(ctx, ctx->cg_rr, CG_MAX_UPDGROUPS * 8));
    CKI(ensure(ctx, ctx->cg_scal, (CG_NSLOT + 5) * 8));
    return IBSN_OK;
}

int run_hvp(ibsn_ctx *ctx, const ibsn_csr *c, const double *a, double eta, double shift,
            const double *v, double *y)
{
    const GatherPlan g = gather_plan(c->m, c->n, c->nnz, c->istar, ctx->num_cus, ctx->max_lds);
    CKH(launch_hvp(g, csr_view(c), a, eta, shift, v, y, P<double>(ctx->cg_au),
                   P<double>(ctx->cg_star), ctx->stream));
    return IBSN_OK;
}

// CG for (H_rho + shift I) x = rhs from 0; result in ctx->cg_x; *iters on host.
// Iterations are enqueued in chunks; after each chunk one small kernel records the
// state, which is copied to pinned host memory behind an event.  The next chunk is
// enqueued before the host waits for the previous record, so the device does not idle
// while the host reads it: the chunk's length is what the residual's observed rate of
// decrease predicts is still needed beyond the iterations already queued.  Iterations
// enqueued after CG has finished are no-ops on the device (they see the done flag and
// carry the final state forward), so overshoot costs only their launches.
int run_cg(ibsn_ctx *ctx, const ibsn_csr *c, const double *a, double eta, double shift,
           const double *rhs, double tol, int maxit, int *iters)
{
    hipStream_t st = ctx->stream;
    CKI(ensure_cg(ctx, c->m, c->n));
    CgState s;
    s.x = P<double>(ctx->cg_x);
    s.r = P<double>(ctx->cg_r);
    s.r2 = P<double>(ctx->cg_r2);
    s.p = P<double>(ctx->cg_p);
    s.Ap = P<double>(ctx->cg_Ap);
    s.au = P<double>(ctx->cg_au);
    s.star_part = P<double>(ctx->cg_star);
    s.pap_part = P<double>(ctx->cg_pap);
    s.rr_part = P<double>(ctx->cg_rr);
    s.scal = P<double>(ctx->cg_scal);
    const CsrView cv = csr_view(c);
    KTimer kt(ctx, IBSN_KT_CG);
    // one workgroup: forced, or automatic for a small factor whose vectors fit in LDS
    const bool single_fits = cg_single_fits(c->m, c->n, ctx->max_lds);
    if (ctx->cg_mode == IBSN_CG_SINGLE ||
        (ctx->cg_mode == IBSN_CG_AUTO && single_fits && c->m <= CG_SINGLE_MAX_DIM &&
         c->n <= CG_SINGLE_MAX_DIM &&
         (double)c->nnz <= CG_SINGLE_ENTRIES_PER_LINE * (double)std::max(c->m, c->n))) {
        if (!single_fits)
            return fail(ctx, IBSN_ERR_UNSUPPORTED,
                        "cg: one-workgroup CG needs n <= %d and (m + n) doubles of LDS",
                        CG_SINGLE_MAX_COLS_PER_THREAD * 1024);
        CKH(launch_cg_single(cv, a, eta, shift, rhs, tol, maxit, s, st));
        double *h = ctx->cg_host;
        CKH(hipMemcpyAsync(h, s.scal, sizeof(double) * CG_NSLOT, hipMemcpyDeviceToHost, st));
        CKH(hipStreamSynchronize(st));
        *iters = (int)h[CG_IT0];
        return IBSN_OK;
    }
    // the barrier counter counts (2 maxit + 1) grids of arrivals in 32 bits
    const bool fits = (2.0 * maxit + 1.0) * CG_PERSIST_MAX_GRID < 4294967295.0;
    const bool coop_ok = ctx->coop && !ctx->coop_off && fits;
    if (ctx->cg_mode == IBSN_CG_PIPE && !coop_ok)
        return fail(ctx, IBSN_ERR_UNSUPPORTED,
                    "cg: the one-barrier CG needs cooperative launches and maxit < 2^21");
    if (coop_ok && (ctx->cg_mode == IBSN_CG_PIPE || ctx->cg_mode == IBSN_CG_AUTO)) {
        // M = P'^T diag(a) P' (c->m2 entries, known from the sparsify pass): the one-barrier
        // form if it stays within CG_PIPE_MAX_RATIO times the factor (always when asked for)
        const int64_t n = c->n, total = c->m2;
        const int lanes = cg_pipe_lanes(n, total);
        int blocks = ctx->cg_blocks;
        if (blocks <= 0) {
            const int64_t per = 2 * (256 / lanes);   // two sweeps of rows per workgroup
            const int64_t g = (n + per - 1) / per;
            blocks = (int)std::min<int64_t>(g, ctx->num_cus);
        }
        blocks = std::max(1, std::min(blocks, CG_PERSIST_MAX_GRID));
        const bool rows_fit = cg_pipe_rows(n, blocks, lanes) <= CG_PIPE_MAX_ROWS;
        if (ctx->cg_mode == IBSN_CG_PIPE && !rows_fit)
            return fail(ctx, IBSN_ERR_UNSUPPORTED, "cg: the one-barrier CG takes at most %d "
                        "rows per lane group (n=%lld on %d workgroups)", CG_PIPE_MAX_ROWS,
                        (long long)n, blocks);
        // a workgroup's entry offsets into M are 32-bit
        if (ctx->cg_mode == IBSN_CG_PIPE && total > (int64_t)INT32_MAX)
            return fail(ctx, IBSN_ERR_UNSUPPORTED, "cg: the one-barrier CG holds at most "
                        "2^31 - 1 entries of P'^T diag(a) P' (%lld here)", (long long)total);
        if (rows_fit && total <= (int64_t)INT32_MAX && (ctx->cg_mode == IBSN_CG_PIPE ||
                         (double)total <= CG_PIPE_MAX_RATIO * (double)c->nnz + (double)n)) {
            CKI(ensure(ctx, ctx->cg_mcnt, (size_t)n * 8));
            CKI(ensure(ctx, ctx->cg_mptr, ((size_t)n + 1) * 8));
            int64_t *mptr = P<int64_t>(ctx->cg_mptr);
            CKH(launch_m_count(cv, P<int64_t>(ctx->cg_mcnt), mptr, st));
            CKI(ensure(ctx, ctx->cg_mcol, (size_t)std::max<int64_t>(total, 1) * 4));
            CKI(ensure(ctx, ctx->cg_mval, (size_t)std::max<int64_t>(total, 1) * 8));
            CKI(ensure(ctx, ctx->cg_w, (size_t)n * 16));
            CKH(launch_m_fill(cv, a, mptr, P<int32_t>(ctx->cg_mcol), P<double>(ctx->cg_mval),
                              st));
            CKI(ensure(ctx, ctx->cg_pp, CG_PIPE_SCRATCH(blocks) * 8));
            double *pp = P<double>(ctx->cg_pp);
            CKH(launch_cg_pipe(blocks, lanes, cv, c->istar, a, mptr, P<int32_t>(ctx->cg_mcol),
                               P<double>(ctx->cg_mval), rhs, eta, shift, tol, maxit, s,
                               P<double>(ctx->cg_w), pp, st));
            double *h = ctx->cg_host;
            CKH(hipMemcpyAsync(h, s.scal, sizeof(double) * CG_NSLOT, hipMemcpyDeviceToHost, st));
            CKH(hipMemcpyAsync(h + CG_NSLOT, pp + 6 * (int64_t)blocks, sizeof(double),
                               hipMemcpyDeviceToHost, st));
            CKH(hipStreamSynchronize(st));
            unsigned flag[2];
            memcpy(flag, h + CG_NSLOT, sizeof(flag));
            if (flag[1] != 0u)
                return fail(ctx, IBSN_ERR_HIP, "cg: a grid barrier of the one-barrier CG timed "
                                               "out (%d workgroups)", blocks);
            *iters = (int)h[CG_IT0];
            return IBSN_OK;
        }
    }
    if (ctx->cg_mode != IBSN_CG_LAUNCHES && coop_ok) {
        // one cooperative launch runs every iteration; one copy of its end state
        const CgPersistPlan pl =
            cg_persist_plan(c->m, c->n, c->nnz, c->istar, ctx->num_cus, ctx->cg_blocks);
        CKI(ensure(ctx, ctx->cg_pp, CG_PERSIST_SCRATCH(pl.blocks) * 8));
        double *pp = P<double>(ctx->cg_pp);
        CKH(launch_cg_persist(pl, cv, a, eta, shift, rhs, tol, maxit, s, pp, st));
        double *h = ctx->cg_host;
        CKH(hipMemcpyAsync(h, s.scal, sizeof(double) * CG_NSLOT, hipMemcpyDeviceToHost, st));
        CKH(hipMemcpyAsync(h + CG_NSLOT, pp + 5 * (int64_t)pl.blocks, sizeof(double),
                           hipMemcpyDeviceToHost, st));
        CKH(hipStreamSynchronize(st));
        unsigned flag[2];
        memcpy(flag, h + CG_NSLOT, sizeof(flag));
        if (flag[1] != 0u)
            return fail(ctx, IBSN_ERR_HIP, "cg: a grid barrier of the one-launch CG timed out "
                                           "(%d workgroups)", pl.blocks);
        *iters = (int)h[CG_IT0];
        return IBSN_OK;
    }
    if (ctx->cg_mode == IBSN_CG_PERSISTENT && !ctx->coop_off)
        return fail(ctx, IBSN_ERR_UNSUPPORTED,
                    "cg: one-launch CG needs cooperative launches and maxit < 2^21");
    const GatherPlan g = gather_plan(c->m, c->n, c->nnz, c->istar, ctx->num_cus, ctx->max_lds);
    CKH(launch_cg_init(c->n, rhs, tol, maxit, s, st));
    int launched = 0;
    // outstanding state records, oldest first: host buffer index and iteration count
    int pend_buf[2], pend_at[2], npend = 0, nextbuf = 0;
    auto enqueue = [&](int chunk) -> int {
        for (int q = 0; q < chunk && launched < maxit; ++q, ++launched)
            CKH(launch_cg_iteration(g, cv, a, eta, shift, s, launched, st));
        CKH(launch_cg_check(g, s, launched, c->n, st));
        double *h = ctx->cg_host + nextbuf * CG_NSLOT;
        CKH(hipMemcpyAsync(h, s.scal, sizeof(double) * CG_NSLOT, hipMemcpyDeviceToHost, st));
        CKH(hipEventRecord(ctx->cg_ev[nextbuf], st));
        pend_buf[npend] = nextbuf;
        pend_at[npend] = launched;
        ++npend;
        nextbuf ^= 1;
        return IBSN_OK;
    };
    CKI(enqueue(8));
    if (launched < maxit)
        CKI(enqueue(4));
    double last_res = -1.0;
    int last_at = 0;
    for (;;) {
        const int b = pend_buf[0], at = pend_at[0];
        pend_buf[0] = pend_buf[1];
        pend_at[0] = pend_at[1];
        --npend;
        CKH(hipEventSynchronize(ctx->cg_ev[b]));
        const double *hs = ctx->cg_host + b * CG_NSLOT;
        const int slot = at & 1;
        if (hs[CG_DONE0 + slot] != 0.0 || at >= maxit) {
            *iters = (int)hs[CG_IT0 + slot];
            break;   // a chunk still queued runs as no-ops
        }
        const double res = std::sqrt(hs[CG_RR0 + slot]);
        int need = 8;   // iterations still needed after `at` (no rate known yet: 8)
        if (last_res > 0.0 && res < last_res && res > tol && tol > 0.0) {
            const double rate = std::log(res / last_res) / (double)(at - last_at);
            need = (int)std::ceil(std::log(tol / res) / rate) + 1;
        }
        last_res = res;
        last_at = at;
        const int queued = (npend > 0 ? pend_at[npend - 1] : at) - at;
        int more = need - queued;
        if (npend == 0)
            more = std::max(more, 2);   // nothing queued: keep going
        if (more > 0 && launched < maxit)
            CKI(enqueue(std::max(2, std::min(more, 64))));
    }
    return IBSN_OK;
}

// Tile search for the dense passes (see ibsn_autotune): the first subproblem's state at
// gamma = 0, every compiled light tile that holds the row timed on eval + stop test and
// every heavy tile on trial + sparsify kernel, for grids of 1, 2 and 4 workgroups per CU;
// the fastest light and heavy tile per grid, then the fastest grid.  A candidate whose
// launch the runtime refuses (its LDS does not fit) is skipped.
int tune_plan(ibsn_ctx *ctx, const ibsn_problem *p, RowPlan *best, double ms[4])
{
    hipStream_t st = ctx->stream;
    const int64_t m = p->m, n = p->n;
    const int mixed = p->precision == IBSN_PREC_MIXED ? 1 : 0;
    RowPlan base;
    if (!plan_rows(m, n, p->cost_kind, ctx->num_cus, &base))
        return fail(ctx, IBSN_ERR_UNSUPPORTED, "no row tile for n=%lld", (long long)n);
    int lt[16][3], ht[16][3];
    const int nl = tile_candidates(n, p->cost_kind, false, lt, 16);
    const int nh = tile_candidates(n, p->cost_kind, true, ht, 16);
    int grids[3], ng = 0;
    for (int per : {1, 2, 4}) {
        const int g = (int)std::min<int64_t>((int64_t)ctx->num_cus * per, m);
        if (ng == 0 || grids[ng - 1] != g)
            grids[ng++] = g;
    }
    RowPlan big = base;
    big.grid = std::max(base.grid, grids[ng - 1]);
    CKI(ensure_ws(ctx, p, big));
    for (DevBuf *b : {&ctx->sv_r, &ctx->sv_M, &ctx->sv_S, &ctx->sv_Mt, &ctx->sv_St})
        CKI(ensure(ctx, *b, m * 8));
    for (DevBuf *b : {&ctx->sv_s, &ctx->sv_g, &ctx->sv_c, &ctx->sv_gv, &ctx->sv_ct, &ctx->sv_gt,
                      &ctx->sv_D})
        CKI(ensure(ctx, *b, n * 8));
    double *r = P<double>(ctx->sv_r), *s = P<double>(ctx->sv_s), *gamma = P<double>(ctx->sv_g);
    double *M = P<double>(ctx->sv_M), *S = P<double>(ctx->sv_S), *Mt = P<double>(ctx->sv_Mt);
    double *St = P<double>(ctx->sv_St), *c = P<double>(ctx->sv_c), *g = P<double>(ctx->sv_gv);
    double *ct = P<double>(ctx->sv_ct), *gt = P<double>(ctx->sv_gt), *D = P<double>(ctx->sv_D);
    double *scal = P<double>(ctx->scal);
    if (!ctx->solver_csr) {
        ctx->solver_csr = new ibsn_csr();
        ctx->solver_csr->ctx = ctx;
    }
    ibsn_csr *csr = ctx->solver_csr;
    CKI(csr_alloc(ctx, csr, m, n));
    CKH(sk_problem_scalars(m, n, p->a, p->b, scal, P<int>(csr->istar_dev), st));
    CKH(sk_dot_slot(m, p->a, p->a, SC_AA, scal, st));
    CKH(sk_dot_slot(n, p->b, p->b, SC_BB, scal, st));
    CKH(sk_init_center(m, n, p->a, p->b, r, s, st));
    CKH(sk_fill(n, 0.0, gamma, st));
    CKH(sk_fill(n, 0.0, D, st));
    CKH(sk_cost_max(m, n, p->ldc, p->cost_kind, p->C, p->y, p->cost_scale,
                    P<double>(ctx->rowpart2), big.grid, scal, st));
    CKH(sk_wmax(n, s, gamma, p->eta, scal, st));
    CKI(read_scal(ctx));
    const double q = quantum_of(ctx->host_scal[SC_WMAX] + ctx->host_scal[SC_CMAX] / p->eta);
    CKH(launch_make_w(s, gamma, q, p->eta, n, lo_split(ctx, p), P<double>(ctx->w),
                      P<double>(ctx->wlo), st));
    const DenseArgs d = dense_args(ctx, p, 0, q, mixed);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CKH(hipEventCreate(&e0));
    CKH(hipEventCreate(&e1));
    // ms per call of fn (three calls after one untimed), or infinity if a launch fails
    auto timed = [&](auto &&fn) -> double {
        if (fn() != IBSN_OK || hipStreamSynchronize(st) != hipSuccess) {
            (void)hipGetLastError();
            return INFINITY;
        }
        (void)hipEventRecord(e0, st);
        for (int k = 0; k < 3; ++k)
            if (fn() != IBSN_OK) {
                (void)hipStreamSynchronize(st);
                (void)hipGetLastError();
                return INFINITY;
            }
        (void)hipEventRecord(e1, st);
        float t = 0.0f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            return INFINITY;
        return (double)t / 3.0;
    };
    auto light_ms = [&](const RowPlan &rp) -> double {
        const double te = timed([&]() {
            return run_eval(ctx, p, rp, 0, q, nullptr, nullptr, M, S, nullptr, c, g, nullptr,
                            mixed);
        });
        // the stop test (both passes, light tile) at the state the eval left
        const double ts = std::isfinite(te) ? timed([&]() {
            return run_stop(ctx, p, rp, 0, q, gamma, M, S, nullptr);
        }) : INFINITY;
        return te + ts;
    };
    auto heavy_ms = [&](const RowPlan &rp) -> double {
        if (run_eval(ctx, p, base, 0, q, nullptr, nullptr, M, S, nullptr, c, g, nullptr, mixed) !=
            IBSN_OK)
            return INFINITY;
        const double tt = timed([&]() {
            return run_trial(ctx, p, rp, 0, q, M, D, 1.0, Mt, St, ct, gt, mixed);
        });
        const double tsp = std::isfinite(tt) ? timed([&]() -> int {
            CKH(launch_sparsify(rp, d, M, S, 1e-3, P<int>(csr->istar_dev), P<int32_t>(csr->col),
                                csr->val.p, P<int32_t>(csr->len), P<double>(ctx->colpart), st));
            return IBSN_OK;
        }) : INFINITY;
        return tt + tsp;
    };
    double best_t = INFINITY;
    *best = base;
    ms[0] = light_ms(base);
    ms[1] = heavy_ms(base);
    ms[2] = ms[0];
    ms[3] = ms[1];
    for (int gi = 0; gi < ng; ++gi) {
        RowPlan rp = base;
        rp.grid = grids[gi];
        double bl = INFINITY, bh = INFINITY;
        RowPlan cand = rp;
        for (int k = 0; k < nl; ++k) {
            RowPlan t = rp;
            t.nt = lt[k][0];
            t.q = lt[k][1];
            t.qf = lt[k][2];
            const double v = light_ms(t);
            if (v < bl) {
                bl = v;
                cand.nt = t.nt;
                cand.q = t.q;
                cand.qf = t.qf;
            }
        }
        for (int k = 0; k < nh; ++k) {
            RowPlan t = rp;
            t.nt_h = ht[k][0];
            t.q_h = ht[k][1];
            t.qf_h = ht[k][2];
            const double v = heavy_ms(t);
            if (v < bh) {
                bh = v;
                cand.nt_h = t.nt_h;
                cand.q_h = t.q_h;
                cand.qf_h = t.qf_h;
            }
        }
        if (bl + bh < best_t) {
            best_t = bl + bh;
            *best = cand;
            ms[2] = bl;
            ms[3] = bh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!std::isfinite(best_t))
        return fail(ctx, IBSN_ERR_HIP, "autotune: no tile could be launched for n=%lld",
                    (long long)n);
    return IBSN_OK;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

// =================================================================================
// exported API
// =================================================================================
namespace ibsn {
hipStream_t ctx_stream(const ibsn_ctx *ctx) { return ctx->stream; }
int ctx_device(const ibsn_ctx *ctx) { return ctx->device; }
int ctx_fail(ibsn_ctx *ctx, int code, const char *msg) { return fail(ctx, code, "%s", msg); }
}  // namespace ibsn

extern "C" {

int ibsn_create(ibsn_ctx **out, int device, void *hip_stream)
{
    if (!out)
        return IBSN_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return IBSN_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess)
        return IBSN_ERR_HIP;
    if (device >= 64)
        return IBSN_ERR_UNSUPPORTED;
    double *scr = nullptr;
    {
        // once per device, with the device current: the address of its copy of `scratch`
        std::lock_guard<std::mutex> lk(scratch_mu);
        if (!scratch_dev[device]) {
            void *ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
                return IBSN_ERR_HIP;
            scratch_dev[device] = (double *)ptr;
        }
        scr = scratch_dev[device];
    }
    ibsn_ctx *ctx = new ibsn_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->scratch = scr;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        ctx->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        ctx->max_lds = prop.sharedMemPerBlock;
    }
    if (hipHostMalloc((void **)&ctx->host_scal, sizeof(double) * (SC_NSLOT + 16)) != hipSuccess) {
        delete ctx;
        return IBSN_ERR_HIP;
    }
    int coop = 0;
    ctx->coop = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) ==
                    hipSuccess && coop != 0;
    if (hipHostMalloc((void **)&ctx->cg_host, sizeof(double) * (2 * CG_NSLOT + 1)) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->cg_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->cg_ev[1], hipEventDisableTiming) != hipSuccess) {
        ibsn_destroy(ctx);
        return IBSN_ERR_HIP;
    }
    *out = ctx;
    return IBSN_OK;
}

void ibsn_destroy(ibsn_ctx *ctx)
{
    if (!ctx)
        return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream)
        (void)hipStreamSynchronize(ctx->stream);
    else
        (void)hipDeviceSynchronize();
    if (ctx->solver_csr) {
        csr_release(ctx->solver_csr);
        delete ctx->solver_csr;
    }
    // handles still open lose their device memory now; ibsn_csr_free later frees the rest
    for (ibsn_csr *c : ctx->csrs) {
        csr_release(c);
        c->ctx = nullptr;
    }
    ctx->csrs.clear();
    DevBuf *bufs[] = {&ctx->w, &ctx->wlo, &ctx->lcv, &ctx->clpart, &ctx->colpart, &ctx->colpart2, &ctx->rowpart, &ctx->rowpart2,
                      &ctx->scal, &ctx->colv, &ctx->cvec, &ctx->gvec, &ctx->yv, &ctx->ecv,
                      &ctx->psiv, &ctx->zv, &ctx->erv, &ctx->zgv, &ctx->stopout, &ctx->tauv,
                      &ctx->cg_x, &ctx->cg_r, &ctx->cg_r2,
                      &ctx->cg_p,
                      &ctx->cg_Ap, &ctx->cg_au, &ctx->cg_star, &ctx->cg_pap, &ctx->cg_rr,
                      &ctx->cg_scal, &ctx->cg_pp, &ctx->sv_r, &ctx->sv_s, &ctx->sv_g, &ctx->sv_M,
                      &ctx->sv_S, &ctx->sv_Mt, &ctx->sv_St, &ctx->sv_ct, &ctx->sv_gt, &ctx->sv_D,
                      &ctx->sv_c, &ctx->sv_gv, &ctx->wd_M, &ctx->wd_S, &ctx->wd_f, &ctx->wd_rr,
                      &ctx->wd_len, &ctx->cg_mcnt, &ctx->cg_mptr, &ctx->cg_mcol, &ctx->cg_mval,
                      &ctx->cg_w};
    for (DevBuf *b : bufs)
        release(*b);
    if (ctx->host_scal)
        (void)hipHostFree(ctx->host_scal);
    if (ctx->cg_host)
        (void)hipHostFree(ctx->cg_host);
    for (hipEvent_t e : ctx->cg_ev)
        if (e)
            (void)hipEventDestroy(e);
    drain_events(ctx);
    for (hipEvent_t e : ctx->ev_free)
        (void)hipEventDestroy(e);
    delete ctx;
}

int ibsn_kernel_timing(ibsn_ctx *ctx, int enable)
{
    if (!ctx)
        return IBSN_ERR_INVALID_ARG;
    CKH(hipSetDevice(ctx->device));
    drain_events(ctx);
    ctx->timing = enable != 0;
    for (int k = 0; k < IBSN_KT_N; ++k) {
        ctx->kt_ms[k] = 0.0;
        ctx->kt_count[k] = 0;
    }
    return IBSN_OK;
}

int ibsn_kernel_times_get(ibsn_ctx *ctx, ibsn_kernel_times *out)
{
    if (!ctx || !out)
        return IBSN_ERR_INVALID_ARG;
    CKH(hipSetDevice(ctx->device));
    drain_events(ctx);
    for (int k = 0; k < IBSN_KT_N; ++k) {
        out->ms[k] = ctx->kt_ms[k];
        out->count[k] = ctx->kt_count[k];
    }
    return IBSN_OK;
}

const char *ibsn_last_error(const ibsn_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int ibsn_num_cus(const ibsn_ctx *ctx) { return ctx ? ctx->num_cus : 0; }

int ibsn_autotune(ibsn_ctx *ctx, const ibsn_problem *prob, ibsn_tile *out)
{
    if (!ctx)
        return IBSN_ERR_INVALID_ARG;
    if (!prob) {
        ctx->tuned.clear();
        return IBSN_OK;
    }
    CKI(check_problem(ctx, prob));
    if (split_width(ctx, prob))
        return fail(ctx, IBSN_ERR_UNSUPPORTED, "autotune: rows split into column blocks "
                    "(n=%lld) run on the built-in tiles", (long long)prob->n);
    if (hipSetDevice(ctx->device) != hipSuccess)
        return fail(ctx, IBSN_ERR_HIP, "autotune: hipSetDevice failed");
    // a shape tuned before is tuned again (the search runs on the default plan)
    const int mixed = prob->precision == IBSN_PREC_MIXED ? 1 : 0;
    std::vector<ibsn_ctx::Tuned> keep;
    for (const auto &t : ctx->tuned)
        if (!(t.m == prob->m && t.n == prob->n && t.kind == prob->cost_kind && t.mixed == mixed))
            keep.push_back(t);
    ctx->tuned.swap(keep);
    RowPlan best;
    double ms[4];
    CKI(tune_plan(ctx, prob, &best, ms));
    ctx->tuned.push_back({prob->m, prob->n, prob->cost_kind, mixed, best});
    if (out) {
        out->nt = best.nt;
        out->q = best.q;
        out->qf = best.qf;
        out->nt_h = best.nt_h;
        out->q_h = best.q_h;
        out->qf_h = best.qf_h;
        out->grid = best.grid;
        out->reserved = 0;
        out->default_light_ms = ms[0];
        out->default_heavy_ms = ms[1];
        out->light_ms = ms[2];
        out->heavy_ms = ms[3];
    }
    return IBSN_OK;
}

int ibsn_set_cg_kernel(ibsn_ctx *ctx, int mode, int blocks)
{
    if (!ctx)
        return IBSN_ERR_INVALID_ARG;
    if (mode < IBSN_CG_AUTO || mode > IBSN_CG_PIPE || blocks < 0 ||
        blocks > CG_PERSIST_MAX_GRID)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "set_cg_kernel: mode 0..4, 0 <= blocks <= %d",
                    CG_PERSIST_MAX_GRID);
    if ((mode == IBSN_CG_PERSISTENT || mode == IBSN_CG_PIPE) && !ctx->coop)
        return fail(ctx, IBSN_ERR_UNSUPPORTED, "set_cg_kernel: no cooperative launches");
    ctx->cg_mode = mode;
    ctx->cg_blocks = blocks;
    return IBSN_OK;
}

int ibsn_set_row_split(ibsn_ctx *ctx, int64_t cols)
{
    if (!ctx)
        return IBSN_ERR_INVALID_ARG;
    if (cols != 0 && (cols < 256 || cols % 64 != 0 || cols > IBSN_MAX_N_F64))
        return fail(ctx, IBSN_ERR_INVALID_ARG,
                    "set_row_split: 0, or a multiple of 64 in [256, %d]", IBSN_MAX_N_F64);
    ctx->split_cols = cols;
    return IBSN_OK;
}

int ibsn_set_csc_fill(ibsn_ctx *ctx, int mode)
{
    static_assert(IBSN_CSC_AUTO == CSC_FILL_AUTO && IBSN_CSC_ENTRY == CSC_FILL_ENTRY &&
                      IBSN_CSC_BLOCK == CSC_FILL_BLOCK,
                  "fill modes of the ABI and the kernels");
    if (!ctx)
        return IBSN_ERR_INVALID_ARG;
    if (mode != IBSN_CSC_AUTO && mode != IBSN_CSC_ENTRY && mode != IBSN_CSC_BLOCK)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "set_csc_fill: IBSN_CSC_AUTO, IBSN_CSC_ENTRY or "
                                               "IBSN_CSC_BLOCK");
    ctx->csc_fill = mode;
    return IBSN_OK;
}

void ibsn_default_options(ibsn_options *o)
{
    if (!o)
        return;
    o->sigma_armijo = 1e-4;
    o->beta = 0.8;
    o->sinkhorn_tol = 1e-3;
    o->sinkhorn_maxit = 10000;
    o->mu0 = 1e-4;
    o->mu_floor = 1e-11;
    o->gap_tol = 1e-8;
    o->marg_tol = 1e-9;
    o->kkt_tol = 0.0;
    o->max_outer = 300;
    o->max_newton = 1000;
    o->max_backtrack = 60;
    o->cg_maxit = 0;
    o->cg_forcing_max = 0.1;
    o->rho_mode = 0;
    o->cg_rtol_min = 1e-6;
    o->stall_limit = 1;
    o->eot = 0;
    o->eot_tol = 1e-9;
    o->mixed_switch = 64.0;
    o->trace = nullptr;
    o->trace_cap = 0;
    o->armijo_warm = 1;
}

int ibsn_center_init(ibsn_ctx *ctx, const ibsn_problem *prob, double *r, double *s)
{
    CKI(check_problem(ctx, prob));
    if (!r || !s)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "r and s are required");
    CKH(hipSetDevice(ctx->device));
    CKH(sk_init_center(prob->m, prob->n, prob->a, prob->b, r, s, ctx->stream));
    return IBSN_OK;
}

int ibsn_center_quantum(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
                        const double *gamma, double *quantum_host)
{
    CKI(check_problem(ctx, prob));
    if (!ctr || !ctr->s || ctr->k < 0 || !gamma || !quantum_host)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "center (k >= 0, s), gamma and output required");
    CKH(hipSetDevice(ctx->device));
    RowPlan rp;
    CKI(plan_for(ctx, prob, &rp));
    CKI(ensure_ws(ctx, prob, rp));
    double *scal = P<double>(ctx->scal);
    CKH(sk_cost_max(prob->m, prob->n, prob->ldc, prob->cost_kind, prob->C, prob->y, prob->cost_scale,
                    P<double>(ctx->rowpart2), rp.grid, scal, ctx->stream));
    CKH(sk_wmax(prob->n, ctr->s, gamma, prob->eta, scal, ctx->stream));
    CKI(read_scal(ctx));
    if (!std::isfinite(ctx->host_scal[SC_CMAX]))
        return fail(ctx, IBSN_ERR_NUMERIC, "C has a NaN or infinite entry");
    const double sigma = (double)(ctr->k + 1) / prob->eta;
    *quantum_host = quantum_of(ctx->host_scal[SC_WMAX] + sigma * ctx->host_scal[SC_CMAX]);
    return IBSN_OK;
}

int ibsn_subproblem_eval(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
                         const double *gamma, double *M, double *S, double *lse, double *colmarg,
                         double *grad, double *obj_host, double *plan)
{
    CKI(check_problem(ctx, prob));
    CKI(check_center(ctx, ctr));
    if (!gamma || !M || !S || !colmarg || !grad)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "gamma, M, S, colmarg and grad are required");
    if (obj_host && !ctr->r)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "the objective needs the centre's r");
    CKH(hipSetDevice(ctx->device));
    RowPlan rp;
    CKI(plan_for(ctx, prob, &rp));
    CKI(ensure_ws(ctx, prob, rp));
    CKH(launch_make_w(ctr->s, gamma, ctr->quantum, prob->eta, prob->n, lo_split(ctx, prob),
                      P<double>(ctx->w), P<double>(ctx->wlo), ctx->stream));
    CKI(run_eval(ctx, prob, rp, ctr->k, ctr->quantum, obj_host ? ctr->r : nullptr, gamma, M, S,
                 lse, colmarg,
                 grad, plan, prob->precision));
    if (obj_host) {
        CKI(read_scal(ctx));
        *obj_host = ctx->host_scal[SC_OBJ];
    }
    return IBSN_OK;
}

int ibsn_trial(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr, const double *gamma,
               const double *M, const double *Delta, double t, double *dL_host, double *M_new,
               double *S_new, double *colmarg_new, double *grad_new)
{
    CKI(check_problem(ctx, prob));
    CKI(check_center(ctx, ctr));
    if (!gamma || !M || !Delta || !dL_host || !M_new || !S_new || !colmarg_new || !grad_new)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "all arrays of ibsn_trial are required");
    if (!(t > 0.0) || !std::isfinite(t))
        return fail(ctx, IBSN_ERR_INVALID_ARG, "step t=%g must be finite and > 0", t);
    CKH(hipSetDevice(ctx->device));
    RowPlan rp;
    CKI(plan_for(ctx, prob, &rp));
    CKI(ensure_ws(ctx, prob, rp));
    CKH(launch_make_w(ctr->s, gamma, ctr->quantum, prob->eta, prob->n, lo_split(ctx, prob),
                      P<double>(ctx->w), P<double>(ctx->wlo), ctx->stream));
    CKI(run_trial(ctx, prob, rp, ctr->k, ctr->quantum, M, Delta, t, M_new, S_new, colmarg_new,
                  grad_new, prob->precision));
    CKI(read_scal(ctx));
    *dL_host = ctx->host_scal[SC_DL];
    return IBSN_OK;
}

int ibsn_sinkhorn_step(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
                       const double *gamma, const double *M, const double *S,
                       const double *colmarg, double *gamma_out)
{
    CKI(check_problem(ctx, prob));
    CKI(check_center(ctx, ctr));
    if (!gamma || !M || !S || !colmarg || !gamma_out)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "gamma, M, S, colmarg and gamma_out are required");
    CKH(hipSetDevice(ctx->device));
    RowPlan rp;
    CKI(plan_for(ctx, prob, &rp));
    CKI(ensure_ws(ctx, prob, rp));
    hipStream_t st = ctx->stream;
    const int64_t m = prob->m, n = prob->n;
    const int split = lo_split(ctx, prob);
    double *w = P<double>(ctx->w), *wlo = P<double>(ctx->wlo), *lc = P<double>(ctx->lcv);
    double *scal = P<double>(ctx->scal);
    CKH(launch_make_w(ctr->s, gamma, ctr->quantum, prob->eta, n, split, w, wlo, st));
    CKH(sk_sum_parts((int)n, 1, 0, colmarg, 1.0, 0.0, -1, SC_CMIN, 2, scal, st));
    CKI(read_scal(ctx));
    if (ctx->host_scal[SC_CMIN] < 1e-290) {
        const int RB = collse_row_blocks(m, n, COLLSE_MAX_RB);
        double *pm = P<double>(ctx->clpart);
        CKH(launch_collse(dense_args(ctx, prob, ctr->k, ctr->quantum), split, M, S, RB, pm,
                          pm + (size_t)RB * n, lc, st));
    } else {
        CKH(sk_log(n, colmarg, lc, st));
    }
    CKH(sk_sinkhorn_step(n, prob->eta, ctr->quantum, split, prob->b, lc, ctr->s, w, wlo, st));
    CKH(sk_gamma_of(n, prob->eta, w, wlo, ctr->s, gamma_out, st));
    return IBSN_OK;
}

int ibsn_outer_update(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
                      const double *gamma, const double *M, const double *S, double *r_out,
                      double *s_out)
{
    CKI(check_problem(ctx, prob));
    CKI(check_center(ctx, ctr));
    if (!gamma || !M || !S || !r_out || !s_out)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "gamma, M, S, r_out and s_out are required");
    CKH(hipSetDevice(ctx->device));
    RowPlan rp;
    CKI(plan_for(ctx, prob, &rp));
    CKI(ensure_ws(ctx, prob, rp));
    double *w = P<double>(ctx->w), *wlo = P<double>(ctx->wlo);
    CKH(launch_make_w(ctr->s, gamma, ctr->quantum, prob->eta, prob->n, lo_split(ctx, prob), w, wlo,
                      ctx->stream));
    CKH(sk_outer_update(prob->m, prob->n, prob->a, M, S, w, wlo, r_out, s_out, ctx->stream));
    return IBSN_OK;
}

int ibsn_sparsify(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
                  const double *gamma, const double *M, const double *S, double rho,
                  int64_t istar, ibsn_csr **out)
{
    CKI(check_problem(ctx, prob));
    CKI(check_center(ctx, ctr));
    if (!gamma || !M || !S || !out)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "gamma, M, S and out are required");
    if (!(rho >= 0.0) || !std::isfinite(rho))
        return fail(ctx, IBSN_ERR_INVALID_ARG, "rho=%g must be finite and >= 0", rho);
    if (istar >= prob->m)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "istar=%lld >= m", (long long)istar);
    *out = nullptr;
    CKH(hipSetDevice(ctx->device));
    RowPlan rp;
    CKI(plan_for(ctx, prob, &rp));
    CKI(ensure_ws(ctx, prob, rp));
    ibsn_csr *c = new ibsn_csr();
    c->ctx = ctx;
    int rc = csr_alloc(ctx, c, prob->m, prob->n);
    if (rc < 0) {
        csr_release(c);
        delete c;
        return rc;
    }
    if (istar < 0) {
        rc = sk_problem_scalars(prob->m, prob->n, prob->a, prob->b, P<double>(ctx->scal),
                                P<int>(c->istar_dev), ctx->stream) == hipSuccess
                 ? IBSN_OK
                 : fail(ctx, IBSN_ERR_HIP, "argmax a failed");
    } else {
        const int iv = (int)istar;
        rc = hipMemcpyAsync(c->istar_dev.p, &iv, 4, hipMemcpyHostToDevice, ctx->stream) ==
                     hipSuccess
                 ? IBSN_OK
                 : fail(ctx, IBSN_ERR_HIP, "istar copy failed");
        if (rc == IBSN_OK)
            rc = hipStreamSynchronize(ctx->stream) == hipSuccess ? IBSN_OK : IBSN_ERR_HIP;
    }
    if (rc == IBSN_OK) {
        if (launch_make_w(ctr->s, gamma, ctr->quantum, prob->eta, prob->n, lo_split(ctx, prob),
                          P<double>(ctx->w), P<double>(ctx->wlo), ctx->stream) != hipSuccess)
            rc = fail(ctx, IBSN_ERR_HIP, "make_w failed");
    }
    if (rc == IBSN_OK)
        rc = run_sparsify(ctx, prob, rp, ctr->k, ctr->quantum, M, S, rho, c, prob->precision);
    if (rc < 0) {
        csr_release(c);
        delete c;
        return rc;
    }
    ctx->csrs.push_back(c);
    *out = c;
    return IBSN_OK;
}

int ibsn_csr_info(ibsn_ctx *ctx, const ibsn_csr *csr, int64_t *nnz, int64_t *istar)
{
    if (!ctx || !csr)
        return IBSN_ERR_INVALID_ARG;
    if (csr->ctx != ctx)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "the factor belongs to another context");
    if (nnz)
        *nnz = csr->nnz;
    if (istar)
        *istar = csr->istar;
    return IBSN_OK;
}

int ibsn_csr_export(ibsn_ctx *ctx, const ibsn_csr *csr, int64_t *row_ptr, int32_t *col,
                    double *val, double *d)
{
    if (!ctx || !csr || !row_ptr || !col || !val || !d)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "all export buffers are required");
    if (csr->ctx != ctx)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "the factor belongs to another context");
    CKH(hipSetDevice(ctx->device));
    CKH(launch_export_csr(csr->m, csr->n, (const int32_t *)csr->col.p, csr->val.p, csr->f32,
                          (const int32_t *)csr->len.p, row_ptr, col, val, csr->nnz,
                          ctx->stream));
    CKH(hipMemcpyAsync(d, csr->d.p, sizeof(double) * csr->n, hipMemcpyDeviceToDevice,
                       ctx->stream));
    return IBSN_OK;
}

void ibsn_csr_free(ibsn_csr *csr)
{
    if (!csr)
        return;
    if (ibsn_ctx *ctx = csr->ctx) {
        (void)hipSetDevice(ctx->device);
        if (ctx->stream)
            (void)hipStreamSynchronize(ctx->stream);
        auto it = std::find(ctx->csrs.begin(), ctx->csrs.end(), csr);
        if (it != ctx->csrs.end())
            ctx->csrs.erase(it);
        csr_release(csr);
    }
    delete csr;
}

int ibsn_hvp(ibsn_ctx *ctx, const ibsn_csr *csr, const double *a, double eta, double shift,
             const double *v, double *y)
{
    if (!ctx)
        return IBSN_ERR_INVALID_ARG;
    if (!csr || !a || !v || !y)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "csr, a, v and y are required");
    if (csr->ctx != ctx)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "the factor belongs to another context");
    if (!(eta > 0.0) || !std::isfinite(shift))
        return fail(ctx, IBSN_ERR_INVALID_ARG, "eta must be > 0 and shift finite");
    CKH(hipSetDevice(ctx->device));
    CKI(ensure_cg(ctx, csr->m, csr->n));
    return run_hvp(ctx, csr, a, eta, shift, v, y);
}

int ibsn_hvp_noalloc(ibsn_ctx *ctx, const ibsn_csr *csr, const double *a, double eta,
                     double shift, const double *v, double *y)
{
    if (!ctx)
        return IBSN_ERR_INVALID_ARG;
    if (!csr || !a || !v || !y)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "csr, a, v and y are required");
    if (csr->ctx != ctx)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "the factor belongs to another context");
    if (!(eta > 0.0) || !std::isfinite(shift))
        return fail(ctx, IBSN_ERR_INVALID_ARG, "eta must be > 0 and shift finite");
    if (csr->m > IBSN_NOALLOC_MAX_M)
        return fail(ctx, IBSN_ERR_INVALID_ARG,
                    "ibsn_hvp_noalloc: m = %lld exceeds its fixed buffer (m <= %d)",
                    (long long)csr->m, (int)IBSN_NOALLOC_MAX_M);
    if (!ctx->scratch)
        return fail(ctx, IBSN_ERR_HIP, "ibsn_hvp_noalloc: no device buffer for this context");
    const GatherPlan g = gather_plan(csr->m, csr->n, csr->nnz, csr->istar, ctx->num_cus,
                                     ctx->max_lds);
    if (g.nstar > CG_MAX_STAR)
        return fail(ctx, IBSN_ERR_UNSUPPORTED, "dense row split into too many chunks");
    CKH(hipSetDevice(ctx->device));
    // u = a o (P_rho v) and the dense row's partials go to the fixed array; every entry the
    // column gather reads is written by the row gather of this call first
    CKH(launch_hvp(g, csr_view(csr), a, eta, shift, v, y, ctx->scratch,
                   ctx->scratch + IBSN_NOALLOC_MAX_M, ctx->stream));
    return IBSN_OK;
}

int ibsn_cg(ibsn_ctx *ctx, const ibsn_csr *csr, const double *a, double eta, double shift,
            const double *rhs, double tol, int maxit, double *x, int *iters_host)
{
    if (!ctx)
        return IBSN_ERR_INVALID_ARG;
    if (!csr || !a || !rhs || !x)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "csr, a, rhs and x are required");
    if (csr->ctx != ctx)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "the factor belongs to another context");
    if (!(eta > 0.0) || !(shift >= 0.0) || !(tol >= 0.0) || maxit < 0)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "need eta > 0, shift >= 0, tol >= 0, maxit >= 0");
    CKH(hipSetDevice(ctx->device));
    int it = 0;
    CKI(run_cg(ctx, csr, a, eta, shift, rhs, tol, maxit, &it));
    CKH(hipMemcpyAsync(x, ctx->cg_x.p, sizeof(double) * csr->n, hipMemcpyDeviceToDevice,
                       ctx->stream));
    CKH(hipStreamSynchronize(ctx->stream));
    if (iters_host)
        *iters_host = it;
    return IBSN_OK;
}

int ibsn_stop(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr, const double *gamma,
              const double *M, const double *S, double *out_host, double *xhat)
{
    CKI(check_problem(ctx, prob));
    CKI(check_center(ctx, ctr));
    if (!gamma || !M || !S || !out_host)
        return fail(ctx, IBSN_ERR_INVALID_ARG, "gamma, M, S and out_host are required");
    CKH(hipSetDevice(ctx->device));
    RowPlan rp;
    CKI(plan_for(ctx, prob, &rp));
    CKI(ensure_ws(ctx, prob, rp));
    CKH(sk_dot_slot(prob->m, prob->a, nullptr, SC_SUMA, P<double>(ctx->scal), ctx->stream));
    CKH(sk_dot_slot(prob->m, prob->a, prob->a, SC_AA, P<double>(ctx->scal), ctx->stream));
    CKH(sk_dot_slot(prob->n, prob->b, prob->b, SC_BB, P<double>(ctx->scal), ctx->stream));
    CKH(launch_make_w(ctr->s, gamma, ctr->quantum, prob->eta, prob->n, lo_split(ctx, prob),
                      P<double>(ctx->w), P<double>(ctx->wlo), ctx->stream));
    CKI(run_stop(ctx, prob, rp, ctr->k, ctr->quantum, gamma, M, S, xhat));
    CKH(hipMemcpyAsync(out_host, ctx->stopout.p, sizeof(double) * 10, hipMemcpyDeviceToHost,
                       ctx->stream));
    CKH(hipStreamSynchronize(ctx->stream));
    return IBSN_OK;
}

// ---------------------------------------------------------------------------------
// the solver (Algorithm 2)
// ---------------------------------------------------------------------------------
int ibsn_solve(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_options *opt_in,
               double *gamma_io, double *r_io, double *s_io, int64_t *k_io, double *plan_out,
               ibsn_report *rep)
{
    CKI(check_problem(ctx, prob));
    ibsn_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        ibsn_default_options(&opt);
    if (opt.max_outer < 1 || opt.max_newton < 1 || opt.max_backtrack < 0 ||
        !(opt.beta > 0 && opt.beta < 1) || !(opt.sigma_armijo > 0 && opt.sigma_armijo < 1) ||
        (opt.eot != 0 && opt.eot != 1) || (opt.eot && !(opt.eot_tol > 0)) ||
        !(opt.mixed_switch >= 0) || opt.trace_cap < 0 || (opt.trace_cap > 0 && !opt.trace) ||
        (opt.armijo_warm != 0 && opt.armijo_warm != 1))
        return fail(ctx, IBSN_ERR_INVALID_ARG, "invalid options");
    const bool resume = k_io && *k_io > 0;
    if (resume && (!r_io || !s_io))
        return fail(ctx, IBSN_ERR_INVALID_ARG, "resume (k > 0) needs r_io and s_io");
    CKH(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int64_t m = prob->m, n = prob->n;
    const double eta = prob->eta;
    RowPlan rp;
    CKI(plan_for(ctx, prob, &rp));
    CKI(ensure_ws(ctx, prob, rp));
    const int cg_maxit = opt.cg_maxit > 0 ? opt.cg_maxit : (int)std::min<int64_t>(n, 70);

    // solver state buffers (context-owned, grow-only: no allocation once warm)
    DevBuf &rB = ctx->sv_r, &sB = ctx->sv_s, &gB = ctx->sv_g, &MB = ctx->sv_M, &SB = ctx->sv_S,
           &MtB = ctx->sv_Mt, &StB = ctx->sv_St, &ctB = ctx->sv_ct, &gtB = ctx->sv_gt,
           &DB = ctx->sv_D, &cB = ctx->sv_c, &gvB = ctx->sv_gv;
    auto cleanup = [&]() {};
    int rc = IBSN_OK;
#define CKS(call)                  \
    do {                           \
        rc = (call);               \
        if (rc < 0) {              \
            cleanup();             \
            return rc;             \
        }                          \
    } while (0)
#define CKSH(call)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            cleanup();                                                                         \
            return fail(ctx, IBSN_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
        }                                                                                      \
    } while (0)
    CKS(ensure(ctx, rB, m * 8));
    CKS(ensure(ctx, sB, n * 8));
    CKS(ensure(ctx, gB, n * 8));
    CKS(ensure(ctx, MB, m * 8));
    CKS(ensure(ctx, SB, m * 8));
    CKS(ensure(ctx, MtB, m * 8));
    CKS(ensure(ctx, StB, m * 8));
    CKS(ensure(ctx, ctB, n * 8));
    CKS(ensure(ctx, gtB, n * 8));
    CKS(ensure(ctx, DB, n * 8));
    if (!ctx->solver_csr) {
        ctx->solver_csr = new ibsn_csr();
        ctx->solver_csr->ctx = ctx;
    }
    ibsn_csr *csr = ctx->solver_csr;
    CKS(csr_alloc(ctx, csr, m, n));
    double *r = P<double>(rB), *s = P<double>(sB), *gamma = P<double>(gB);
    double *M = P<double>(MB), *S = P<double>(SB), *Mt = P<double>(MtB), *St = P<double>(StB);
    CKS(ensure(ctx, cB, n * 8));
    CKS(ensure(ctx, gvB, n * 8));
    double *c = P<double>(cB), *g = P<double>(gvB);
    double *ct = P<double>(ctB), *gt = P<double>(gtB), *Delta = P<double>(DB);
    double *scal = P<double>(ctx->scal);

    // problem checks and per-problem scalars (istar, sums, a^T a and b^T b)
    CKSH(sk_problem_scalars(m, n, prob->a, prob->b, scal, P<int>(csr->istar_dev), st));
    CKSH(sk_dot_slot(m, prob->a, prob->a, SC_AA, scal, st));
    CKSH(sk_dot_slot(n, prob->b, prob->b, SC_BB, scal, st));
    CKS(read_scal(ctx));
    {
        const double *h = ctx->host_scal;
        const double tol = 1e-12 * (double)std::max(m, n);
        if (h[SC_BAD] != 0.0 || !(h[SC_MINA] > 0.0) || !(h[SC_MINB] > 0.0) ||
            std::fabs(h[SC_SUMA] - 1.0) > tol || std::fabs(h[SC_SUMB] - 1.0) > tol) {
            cleanup();
            return fail(ctx, IBSN_ERR_INVALID_ARG,
                        "marginals must be positive, finite and sum to 1 (sum a=%.17g, sum b=%.17g, "
                        "min a=%g, min b=%g)",
                        h[SC_SUMA], h[SC_SUMB], h[SC_MINA], h[SC_MINB]);
        }
    }
    int64_t k = 0;
    if (resume) {
        k = *k_io;
        CKSH(hipMemcpyAsync(r, r_io, m * 8, hipMemcpyDeviceToDevice, st));
        CKSH(hipMemcpyAsync(s, s_io, n * 8, hipMemcpyDeviceToDevice, st));
    } else if (opt.eot) {
        // (E)IBSN: X^0 = 1 1^T (appendix C.4): the subproblem is entropic OT with cost C
        CKSH(hipMemsetAsync(r, 0, m * 8, st));
        CKSH(hipMemsetAsync(s, 0, n * 8, st));
    } else {
        CKSH(sk_init_center(m, n, prob->a, prob->b, r, s, st));
    }
    if (gamma_io)
        CKSH(hipMemcpyAsync(gamma, gamma_io, n * 8, hipMemcpyDeviceToDevice, st));
    else
        CKSH(hipMemsetAsync(gamma, 0, n * 8, st));
    if (!resume)
        CKSH(sk_center(n, gamma, st));

    // per-problem maximum of |C| (sets the grid spacing of each outer iteration)
    CKSH(sk_cost_max(m, n, prob->ldc, prob->cost_kind, prob->C, prob->y, prob->cost_scale,
                     P<double>(ctx->rowpart2), rp.grid,
                     scal, st));
    CKS(read_scal(ctx));
    const double cmax = ctx->host_scal[SC_CMAX];
    if (!std::isfinite(cmax))
        CKS(fail(ctx, IBSN_ERR_NUMERIC, "C has a NaN or infinite entry"));
    double *w = P<double>(ctx->w), *wlo = P<double>(ctx->wlo), *lc = P<double>(ctx->lcv);
    const int split = lo_split(ctx, prob);
    // Mixed precision: Newton steps run their passes (sparsify, trial) in the FP32 form
    // while ||g||_2 >= mixed_switch * eps32 * ||b||_2; below that, after a mixed-form line
    // search fails, and always for the Sinkhorn steps, the stop test and the outer update,
    // the state comes from FP64 passes (an FP64 eval refreshes a state left by a mixed pass).
    const bool mx_on = prob->precision == IBSN_PREC_MIXED;
    double mx_thr = INFINITY;
    if (mx_on)
        mx_thr = opt.mixed_switch * (double)FLT_EPSILON * std::sqrt(ctx->host_scal[SC_BB]);

    ibsn_report R;
    memset(&R, 0, sizeof(R));
    R.status = IBSN_WARN_MAXITER;
    double nnz_sum = 0.0;
    int64_t nnz_calls = 0;
    const double t0 = now_s();
    double stop_h[10] = {0};
    const int64_t k0 = k;
    const double mn = (double)m * (double)n;
    double t_prev = 1.0;   // step of the last accepted line search (armijo_warm)
    // per-outer-iteration record: the report's counters at the start of the iteration
    ibsn_report Rb;
    double nnz_sum_b = 0.0;
    int64_t nnz_calls_b = 0;
    double t_iter = 0.0;
    auto record = [&](bool inner_stopped) {
        const int64_t idx = k - k0;
        if (idx >= opt.trace_cap)
            return;
        ibsn_iter_record &T = opt.trace[idx];
        memset(&T, 0, sizeof(T));
        T.k = k;
        T.newton = R.newton - Rb.newton;
        T.cg = R.cg - Rb.cg;
        T.sinkhorn = R.sinkhorn - Rb.sinkhorn;
        T.backtracks = R.backtracks - Rb.backtracks;
        T.stop_tests = R.stop_tests - Rb.stop_tests;
        T.passes = R.passes - Rb.passes;
        T.mixed_passes = R.mixed_passes - Rb.mixed_passes;
        T.grad_norm = R.grad_norm;
        T.primal = R.primal;
        T.dual = R.dual;
        T.rel_gap = R.rel_gap;
        T.kkt = R.kkt;
        T.dphi = R.dphi;
        T.marg_l1 = R.marg_l1;
        T.nnz_mean = nnz_calls > nnz_calls_b
                         ? (nnz_sum - nnz_sum_b) / (double)(nnz_calls - nnz_calls_b)
                         : 0.0;
        T.t_eval = R.t_eval - Rb.t_eval;
        T.t_sparsify = R.t_sparsify - Rb.t_sparsify;
        T.t_cg = R.t_cg - Rb.t_cg;
        T.t_linesearch = R.t_linesearch - Rb.t_linesearch;
        T.t_stop = R.t_stop - Rb.t_stop;
        T.t_total = now_s() - t_iter;
        T.inner_stopped = inner_stopped ? 1 : 0;
        R.trace_len = idx + 1;
    };
    for (; k < k0 + opt.max_outer; ++k) {
        Rb = R;
        nnz_sum_b = nnz_sum;
        nnz_calls_b = nnz_calls;
        t_iter = now_s();
        const double mu = std::max(opt.mu0 / ((double)(k + 1) * (double)(k + 1)), opt.mu_floor);
        const double sigma = (double)(k + 1) / eta;
        double ta = now_s();
        // grid of this outer iteration and the potentials w = grid(s + gamma/eta)
        CKSH(sk_wmax(n, s, gamma, eta, scal, st));
        CKS(read_scal(ctx));
        const double q = quantum_of(ctx->host_scal[SC_WMAX] + sigma * cmax);
        CKSH(launch_make_w(s, gamma, q, eta, n, split, w, wlo, st));
        bool state_mx = false;   // (M, S, c, g) come from a mixed-precision pass
        bool fp64_lock = false;  // FP64 passes for the rest of this subproblem
        auto refresh = [&]() -> int {   // FP64 eval at the current point
            CKI(run_eval(ctx, prob, rp, k, q, nullptr, nullptr, M, S, nullptr, c, g, nullptr, 0));
            ++R.passes;
            state_mx = false;
            return read_scal(ctx);
        };
        // fresh evaluation of the new subproblem
        CKS(run_eval(ctx, prob, rp, k, q, nullptr, nullptr, M, S, nullptr, c, g, nullptr,
                     mx_on ? 1 : 0));
        ++R.passes;
        if (mx_on)
            ++R.mixed_passes;
        state_mx = mx_on;
        if (!mx_on)
            CKSH(sk_sum_parts((int)n, 1, 0, c, 1.0, 0.0, -1, SC_CMIN, 2, scal, st));
        CKS(read_scal(ctx));
        if (state_mx && (ctx->host_scal[SC_GN] < mx_thr ||
                         (opt.sinkhorn_maxit > 0 && ctx->host_scal[SC_GN] >= opt.sinkhorn_tol))) {
            CKS(refresh());
            CKSH(sk_sum_parts((int)n, 1, 0, c, 1.0, 0.0, -1, SC_CMIN, 2, scal, st));
            CKS(read_scal(ctx));
        }
        // Sinkhorn warm-up (Algorithm 2, steps 3-4), on the grid potentials
        for (int it = 0; it < opt.sinkhorn_maxit && ctx->host_scal[SC_GN] >= opt.sinkhorn_tol;
             ++it) {
            // lc = log c; in the log domain (column LSE pass) when a column sum is near or
            // below the bottom of the FP64 range
            if (ctx->host_scal[SC_CMIN] < 1e-290) {
                const int RB = collse_row_blocks(m, n, COLLSE_MAX_RB);
                double *pm = P<double>(ctx->clpart);
                CKSH(launch_collse(dense_args(ctx, prob, k, q), split, M, S, RB, pm,
                                   pm + (size_t)RB * n, lc, st));
                ++R.passes;
            } else {
                CKSH(sk_log(n, c, lc, st));
            }
            CKSH(sk_sinkhorn_step(n, eta, q, split, prob->b, lc, s, w, wlo, st));
            CKS(run_eval(ctx, prob, rp, k, q, nullptr, nullptr, M, S, nullptr, c, g, nullptr, 0));
            ++R.passes;
            ++R.sinkhorn;
            CKSH(sk_sum_parts((int)n, 1, 0, c, 1.0, 0.0, -1, SC_CMIN, 2, scal, st));
            CKS(read_scal(ctx));
        }
        if (!std::isfinite(ctx->host_scal[SC_GN])) {
            cleanup();
            return fail(ctx, IBSN_ERR_NUMERIC, "non-finite gradient at outer iteration %lld",
                        (long long)k);
        }
        R.t_eval += now_s() - ta;
        bool stopped = false;
        bool tested = false;   // stop_h holds the stop pass at the current iterate
        int stalls = 0;
        for (int v = 0; v < opt.max_newton; ++v) {
            if (state_mx && (fp64_lock || ctx->host_scal[SC_GN] < mx_thr))
                CKS(refresh());
            const double gn = ctx->host_scal[SC_GN];
            const int mxs = (mx_on && !fp64_lock && gn >= mx_thr) ? 1 : 0;
            if (opt.eot && gn < opt.eot_tol) {   // (E)IBSN: the single subproblem is solved
                stopped = true;
                break;
            }
            const double rho = opt.rho_mode == 1 ? 0.0 : eta * gn / mn;   // step 6
            ta = now_s();
            CKS(run_sparsify(ctx, prob, rp, k, q, M, S, rho, csr, mxs));   // step 7
            ++R.passes;
            R.mixed_passes += mxs;
            R.nnz_last = (double)csr->nnz;
            nnz_sum += (double)csr->nnz;
            ++nnz_calls;
            R.t_sparsify += now_s() - ta;
            ta = now_s();
            CKSH(sk_neg(n, g, Delta, st));   // rhs = -g
            int cgit = 0;
            const double tol = std::max(std::min(opt.cg_forcing_max, gn), opt.cg_rtol_min) * gn;
            CKS(run_cg(ctx, csr, prob->a, eta, gn, Delta, tol, cg_maxit, &cgit));   // step 8
            CKSH(hipMemcpyAsync(Delta, ctx->cg_x.p, n * 8, hipMemcpyDeviceToDevice, st));
            R.cg += cgit;
            R.t_cg += now_s() - ta;
            ta = now_s();
            CKSH(sk_dot_slot(n, g, Delta, SC_GD, scal, st));
            double t = opt.armijo_warm ? std::min(1.0, t_prev / opt.beta) : 1.0;
            int bt = 0;
            bool accepted = false;
            for (;;) {   // step 9: Armijo backtracking on a finite decrease
                CKS(run_trial(ctx, prob, rp, k, q, M, Delta, t, Mt, St, ct, gt, mxs));
                ++R.passes;
                R.mixed_passes += mxs;
                CKS(read_scal(ctx));
                const double gd = ctx->host_scal[SC_GD];
                const double dL = ctx->host_scal[SC_DL];
                // a trial whose gradient is not finite is never accepted
                if (std::isfinite(dL) && std::isfinite(ctx->host_scal[SC_GN]) &&
                    dL <= opt.sigma_armijo * t * gd) {
                    accepted = true;
                    break;
                }
                if (bt >= opt.max_backtrack)
                    break;
                t *= opt.beta;
                ++bt;
            }
            R.backtracks += bt;
            if (!accepted && mxs) {
                // the FP32 form could not certify a decrease: continue in FP64.  The trials
                // overwrote the norms of g; a mixed state is refreshed by an FP64 eval at the
                // top of the loop, an FP64 state gets its own norms back here.
                fp64_lock = true;
                if (!state_mx) {
                    CKSH(sk_gnorms(n, g, scal, st));
                    CKS(read_scal(ctx));
                }
                R.t_linesearch += now_s() - ta;
                continue;
            }
            if (!accepted) {
                // no acceptable step: keep the iterate, restore the norms of its g and
                // end the inner loop
                CKSH(sk_gnorms(n, g, scal, st));
                CKS(read_scal(ctx));
                R.t_linesearch += now_s() - ta;
                break;
            }
            t_prev = t;
            // step 10: w += tau, exactly in the two-level potential (on the grid when the
            // potentials are kept there); the accepted trial is the new iterate
            CKSH(sk_dd_axpy(n, q, P<double>(ctx->tauv), w, wlo, st));
            std::swap(M, Mt);
            std::swap(S, St);
            std::swap(c, ct);
            std::swap(g, gt);
            state_mx = mxs != 0;
            tested = false;
            ++R.newton;
            R.t_linesearch += now_s() - ta;
            // step 12 with the practical schedule: gradient gate, then D_phi test (on an
            // FP64 state)
            if (!opt.eot && state_mx && ctx->host_scal[SC_GN] < mu)
                CKS(refresh());
            if (!opt.eot && ctx->host_scal[SC_GN] < mu) {
                ta = now_s();
                CKSH(sk_gamma_of(n, eta, w, wlo, s, gamma, st));
                CKS(run_stop(ctx, prob, rp, k, q, gamma, M, S, nullptr, c));
                R.passes += 2;
                ++R.stop_tests;
                CKSH(hipMemcpyAsync(stop_h, ctx->stopout.p, sizeof(stop_h), hipMemcpyDeviceToHost,
                                    st));
                CKSH(hipStreamSynchronize(st));
                R.t_stop += now_s() - ta;
                tested = true;
                if (stop_h[0] <= (double)std::min(m, n) * mu) {
                    stopped = true;
                    break;
                }
                if (++stalls >= opt.stall_limit)
                    break;
            }
        }
        if (state_mx)
            CKS(refresh());
        CKSH(sk_gamma_of(n, eta, w, wlo, s, gamma, st));
        // the certificate at the final iterate; when the inner loop ended on a failed test
        // (the stall rule, or a line search that found no step after it) the test already
        // computed it at this iterate
        if ((!stopped && !tested) || opt.eot) {
            ta = now_s();
            CKS(run_stop(ctx, prob, rp, k, q, gamma, M, S, nullptr, c));
            R.passes += 2;
            ++R.stop_tests;
            CKSH(hipMemcpyAsync(stop_h, ctx->stopout.p, sizeof(stop_h), hipMemcpyDeviceToHost, st));
            CKSH(hipStreamSynchronize(st));
            R.t_stop += now_s() - ta;
        }
        const double primal = stop_h[1], dual = stop_h[2];
        R.primal = primal;
        R.dual = dual;
        R.rel_gap = (primal - dual) / std::fabs(primal);
        R.kkt = stop_h[4];
        R.dphi = stop_h[0];
        R.grad_norm = ctx->host_scal[SC_GN];
        R.marg_l1 = ctx->host_scal[SC_G1];
        const bool done = (R.rel_gap <= opt.gap_tol && (opt.marg_tol <= 0 || R.marg_l1 <= opt.marg_tol)) ||
                          (opt.kkt_tol > 0 && R.kkt <= opt.kkt_tol);
        if (opt.eot) {
            // (E)IBSN: one subproblem and no outer update; the centre stays (0, 0)
            if (plan_out) {
                CKS(run_stop(ctx, prob, rp, k, q, gamma, M, S, plan_out, c));
                R.passes += 2;
            }
            R.status = R.grad_norm < opt.eot_tol ? IBSN_OK : IBSN_WARN_MAXITER;
            record(stopped);
            ++k;
            break;
        }
        if (plan_out && (done || k + 1 == k0 + opt.max_outer)) {
            CKS(run_stop(ctx, prob, rp, k, q, gamma, M, S, plan_out, c));
            R.passes += 2;
        }
        // step 13: X^{k+1} = X^{k,v+1}, i.e. r = log a - lse, s = w; k = k+1; gamma kept
        CKSH(sk_outer_update(m, n, prob->a, M, S, w, wlo, r, s, st));
        record(stopped);
        if (done) {
            R.status = IBSN_OK;
            ++k;
            break;
        }
    }
    R.outer = k - k0;
    CKSH(hipStreamSynchronize(st));
    R.t_total = now_s() - t0;
    R.nnz_mean = nnz_calls > 0 ? nnz_sum / (double)nnz_calls : 0.0;
    if (gamma_io)
        CKSH(hipMemcpyAsync(gamma_io, gamma, n * 8, hipMemcpyDeviceToDevice, st));
    if (r_io)
        CKSH(hipMemcpyAsync(r_io, r, m * 8, hipMemcpyDeviceToDevice, st));
    if (s_io)
        CKSH(hipMemcpyAsync(s_io, s, n * 8, hipMemcpyDeviceToDevice, st));
    if (k_io)
        *k_io = k;
    CKSH(hipStreamSynchronize(st));
    if (rep)
        *rep = R;
    cleanup();
    return R.status;
#undef CKS
#undef CKSH
}

int ibsn_solve_batch(ibsn_ctx *const *ctxs, int nctx, int64_t nprob, const ibsn_problem *probs,
                     const ibsn_options *opt, double *const *gamma_io, ibsn_report *reps,
                     int32_t *status)
{
    if (!ctxs || nctx < 1 || nprob < 0 || (nprob > 0 && (!probs || !status)))
        return IBSN_ERR_INVALID_ARG;
    for (int w = 0; w < nctx; ++w) {
        if (!ctxs[w])
            return IBSN_ERR_INVALID_ARG;
        for (int v = 0; v < w; ++v)
            if (ctxs[v] == ctxs[w])
                return fail(ctxs[w], IBSN_ERR_INVALID_ARG, "each worker needs its own context");
    }
    // longest (largest m n) first, then a shared counter: each worker takes the next problem
    std::vector<int64_t> order((size_t)nprob);
    std::iota(order.begin(), order.end(), (int64_t)0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
        return probs[x].m * probs[x].n > probs[y].m * probs[y].n;
    });
    // Several contexts solve at once on their own streams: no cooperative launches there,
    // since a cooperative grid is sized for a device that it has to itself (another
    // stream's kernels may hold the compute units its workgroups wait for).  CG runs in
    // one workgroup where that applies, else as kernel launches.
    for (int w = 0; w < nctx; ++w)
        ctxs[w]->coop_off = nctx > 1;
    std::atomic<int64_t> next{0};
    auto worker = [&](int w) {
        for (;;) {
            const int64_t t = next.fetch_add(1);
            if (t >= nprob)
                break;
            const int64_t i = order[(size_t)t];
            ibsn_report r;
            status[i] = ibsn_solve(ctxs[w], &probs[i], opt, gamma_io ? gamma_io[i] : nullptr,
                                   nullptr, nullptr, nullptr, nullptr, reps ? &reps[i] : &r);
        }
    };
    std::vector<std::thread> pool;
    pool.reserve((size_t)nctx);
    for (int w = 1; w < nctx; ++w)
        pool.emplace_back(worker, w);
    worker(0);
    for (std::thread &t : pool)
        t.join();
    for (int w = 0; w < nctx; ++w)
        ctxs[w]->coop_off = false;
    return IBSN_OK;
}

}  // extern "C"
