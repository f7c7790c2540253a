// dense_stop.hip -- the stop-test passes (Algorithm 3, certificate), the fixed-order column
// reduction and the choice of row tiles, on gfx950; helpers in dense_common.h.
#include "dense_common.h"

namespace ibsn {
namespace {

// ---------------------------------------------------------------------------------
// Stop test pass 1 (Algorithm 3, steps 2-8): X = a_i P; z_i; column sums of X and z X.
// Column block of a split row: the first launch writes the block's row sums of X to rsum
// (column sums of X as usual); the second takes z from zin for the column sums of z X.
// Null outputs are not written.
// ---------------------------------------------------------------------------------
template <int NT, int Q, int QF, int VEC, typename CT, bool SPLIT>
__global__ __launch_bounds__(NT) void k_stop1(const CT *__restrict__ C, int64_t ldc,
                                              const double *__restrict__ py, double pscale, int m, int n,
                                              double sigma, const double *__restrict__ w,
                                              const double *__restrict__ wlo,
                                              const double *__restrict__ a,
                                              const double *__restrict__ M,
                                              const double *__restrict__ S,
                                              double *__restrict__ z, double *__restrict__ colpart,
                                              double *__restrict__ colpart2,
                                              double *__restrict__ rowpart,
                                              double *__restrict__ rsum,
                                              const double *__restrict__ zin)
{
    constexpr int E = Q * VEC;
    constexpr bool LO = lo_tile(NT, Q, VEC);
    using RedSum = BlockRed<NT, OP_SUM>;
    __shared__ double lds[RedSum::LDS];
    __shared__ double rM[ROWCH], rS[ROWCH], rA[ROWCH];
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    extern __shared__ double wl[];   // w staged in LDS (n doubles, then the FP32 low parts)
    __shared__ double etab[EXP_TAB];
    double ax[E], az[E], x[E];
    exp_table_init(etab);
    stage_w2<LO>(w, wlo, n, wl);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        ax[e] = 0.0;
        az[e] = 0.0;
    }
    double rowacc = 0.0;
    row_loop<NT, Q, QF, VEC>(
        C, ldc, py, pscale, n, i0, i1, [&](int i) { stage_rows(i, i1, M, rM, S, rS, a, rA); },
        [&](int i, int slot, const auto *xr) {
            const double Mi = rM[slot], ai = rA[slot], aS = ai / rS[slot];
            double red[1] = {0.0};
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const bool valid = slot_valid<QF, NT, VEC>(e, n);
                const int j = slot_col<QF, NT, VEC>(e, n);
                const double xa = add_lo<LO>(fma(-sigma, (double)xr[e], wl[j] - Mi), wl, n, j);
                const double X = exp_tab_z(valid ? xa : -INFINITY, etab) * aS;
                x[e] = X;
                red[0] += X;
            }
            RedSum::run(red, lds, parity);
            const double rs = red[0];
            const double zi = (SPLIT && zin) ? zin[i] : fmin(ai / rs, 1.0);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                ax[e] += x[e];
                az[e] = fma(zi, x[e], az[e]);
            }
            if (threadIdx.x == 0) {
                if (!SPLIT)
                    z[i] = zi;
                else if (rsum)
                    rsum[i] = rs;
                rowacc += (rs - ai) * (rs - ai);
            }
        });
    if (!SPLIT || colpart)
        store_cols<NT, Q, VEC>(colpart + (int64_t)blockIdx.x * n, n, ax);
    if (!SPLIT || colpart2)
        store_cols<NT, Q, VEC>(colpart2 + (int64_t)blockIdx.x * n, n, az);
    if (!SPLIT && threadIdx.x == 0)
        rowpart[blockIdx.x] = rowacc;
}

// ---------------------------------------------------------------------------------
// Stop test pass 2, in two streaming passes over C (Algorithm 3, steps 9-11, and the
// certificate of appendix C.1).
// Pass 2a, per row: e_r,i = max(a_i - z_i sum_j X_ij y_j, 0) (exactly >= 0; the clamp
// removes rounding), and the c-transforms zg_i = min_j (C_ij - gamma_j),
// zp_i = min_j (C_ij - psi_j); per workgroup sum_i a_i zg_i and sum_i a_i zp_i.
// Column block of a split row (rowred given): the block's sum_j X_ij y_j and the two minima
// go to rowred (three arrays of m) instead, and nothing else is written.
// ---------------------------------------------------------------------------------
template <int NT, int Q, int QF, int VEC, typename CT>
__global__ __launch_bounds__(NT) void k_stop2a(const CT *__restrict__ C, int64_t ldc,
                                              const double *__restrict__ py, double pscale, int m, int n,
                                               double sigma, const double *__restrict__ w,
                                               const double *__restrict__ wlo,
                                               const double *__restrict__ a,
                                               const double *__restrict__ M,
                                               const double *__restrict__ S,
                                               const double *__restrict__ gamma,
                                               const double *__restrict__ psi,
                                               const double *__restrict__ y,
                                               const double *__restrict__ z,
                                               double *__restrict__ er_row,
                                               double *__restrict__ zg_row,
                                               double *__restrict__ rowpart,
                                               double *__restrict__ rowred)
{
    constexpr int E = Q * VEC;
    constexpr bool LO = lo_tile(NT, Q, VEC);
    using Red3 = BlockRed<NT, OP_SUM, OP_MIN, OP_MIN>;
    __shared__ double lds[Red3::LDS];
    extern __shared__ double wl[];   // w staged in LDS (n doubles, then the FP32 low parts)
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    __shared__ double etab[EXP_TAB];
    exp_table_init(etab);
    stage_w2<LO>(w, wlo, n, wl);
    constexpr int RCA = 32;   // rows per staged chunk (static LDS within 3.5 KB)
    __shared__ double rM[RCA], rS[RCA], rA[RCA], rZ[RCA];
    double azg = 0.0, azp = 0.0;
    row_loop<NT, Q, QF, VEC, true, RCA>(
        C, ldc, py, pscale, n, i0, i1, [&](int i) { stage_rows<RCA>(i, i1, M, rM, S, rS, a, rA, z, rZ); },
        [&](int i, int slot, const auto *cst) {
        const double Mi = rM[slot], ai = rA[slot], aS = ai / rS[slot];
        double red[3] = {0.0, INFINITY, INFINITY};
        // column loads kept in the row loop and one entry ahead, as in pass 2b; y only
        // where X_ij > 0 (a few entries per row once the plan is sparse)
        const double *yv = y, *gv = gamma, *pv = psi;
        asm volatile("" : "+s"(yv), "+s"(gv), "+s"(pv));
        int jn = slot_col<QF, NT, VEC>(0, n);
        double ng = gv[jn], np = pv[jn];
#pragma unroll 2
        for (int e = 0; e < E; ++e) {
            const bool valid = slot_valid<QF, NT, VEC>(e, n);
            const int j = jn;
            const double gj = ng, pj = np;
            if (e + 1 < E) {
                jn = slot_col<QF, NT, VEC>(e + 1, n);
                ng = gv[jn];
                np = pv[jn];
            }
            const double c = valid ? (double)cst[e] : 0.0;
            const double Xv =
                exp_tab_z(valid ? add_lo<LO>(fma(-sigma, c, wl[j] - Mi), wl, n, j) : -INFINITY,
                        etab) * aS;
            if (Xv > 0.0)
                red[0] = fma(Xv, yv[j], red[0]);
            red[1] = fmin(red[1], valid ? c - gj : INFINITY);
            red[2] = fmin(red[2], valid ? c - pj : INFINITY);
        }
        Red3::template run_part<0>(red, lds, parity);   // used by thread 0 only
        if (threadIdx.x == 0 && rowred) {
            rowred[i] = red[0];
            rowred[m + i] = red[1];
            rowred[2 * (int64_t)m + i] = red[2];
        } else if (threadIdx.x == 0) {
            er_row[i] = fmax(ai - rZ[slot] * red[0], 0.0);
            zg_row[i] = red[1];
            azg += ai * red[1];
            azp += ai * red[2];
        }
        });
    if (threadIdx.x == 0 && !rowred) {
        double *o = rowpart + (int64_t)blockIdx.x * STOP2_NSLOT;
        o[STOP2_AZG] = azg;
        o[STOP2_AZP] = azp;
    }
}

// Pass 2b, streaming: Xhat = z X y + e_r e_c^T / ||e_r||_1, D_phi(Xhat, X) in the log
// domain (log X_ij = log a_i - log S_i + (theta_ij - M_i)), <C,Xhat>, <C,X>, min Xhat,
// <X, U> with U_ij = C_ij - gamma_j - zg_i, and ||X||_F^2, ||C||_F^2 for Delta_kkt.
// Where X_ij = 0 (all but a few entries of a row once the plan is sparse) Xhat_ij is the
// rank-one term es_i e_c,j, and its D_phi term es_i e_c,j (log es_i + log e_c,j - log X_ij - 1)
// is summed per row from three sums: of e_c,j and of e_c,j log e_c,j over the thread's
// columns (fixed for the kernel, less the row's entries with X_ij > 0) and of e_c,j x_ij.
// No logarithm is then taken per entry, and y and gamma are read only where X_ij > 0.
template <int NT, int Q, int QF, int VEC, typename CT>
__global__ __launch_bounds__(NT) void k_stop2b(const CT *__restrict__ C, int64_t ldc,
                                              const double *__restrict__ py, double pscale, int m, int n,
                                               double sigma, const double *__restrict__ w,
                                               const double *__restrict__ wlo,
                                               const double *__restrict__ a,
                                               const double *__restrict__ M,
                                               const double *__restrict__ S,
                                               const double *__restrict__ gamma,
                                               const double *__restrict__ y,
                                               const double *__restrict__ ec,
                                               const double *__restrict__ z,
                                               const double *__restrict__ er_row,
                                               const double *__restrict__ zg_row,
                                               const double *__restrict__ er1p,
                                               double *__restrict__ xhat,
                                               double *__restrict__ rowpart, int64_t ldx)
{
    constexpr int E = Q * VEC;
    constexpr bool LO = lo_tile(NT, Q, VEC);
    using RedEnd = BlockRed<NT, OP_SUM, OP_SUM, OP_SUM, OP_SUM, OP_MIN, OP_SUM, OP_SUM>;
    __shared__ double lds[RedEnd::LDS1];
    extern __shared__ double wl[];   // w staged in LDS (n doubles, then the FP32 low parts)
    int i0, i1;
    row_range(m, i0, i1);
    __shared__ double etab[EXP_TAB];
    __shared__ __align__(16) double ltab[2 * LOG_TAB];
    log_table_init(ltab);
    exp_table_init(etab);   // its barrier also publishes ltab
    stage_w2<LO>(w, wlo, n, wl);
    // 8 rows per staged chunk: with an n-vector of 20000 doubles the static LDS (exp and log
    // tables, reduction buffer, row scalars: 3328 bytes) must stay within 3.5 KB
    constexpr int RC = 8;
    __shared__ double rM[RC], rS[RC], rA[RC], rZ[RC], rE[RC], rG[RC];
    double t_dphi = 0.0, t_cxh = 0.0, t_cx = 0.0, t_xu = 0.0, t_xhmin = INFINITY, t_xf = 0.0,
           t_cf = 0.0;
    const double er1 = *er1p;   // written by the stop preparation kernel before this one
    const double inv_er1 = er1 > 0.0 ? 1.0 / er1 : 0.0;
    // over this thread's columns (the same in every row): sum e_c,j and sum e_c,j log e_c,j
    double t_sec = 0.0, t_slec = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (slot_valid<QF, NT, VEC>(e, n)) {
            const double v = ec[col_of<NT, VEC>(e)];
            t_sec += v;
            t_slec += v > 0.0 ? v * log_tab(v, ltab) : 0.0;
        }
    }
    row_loop<NT, Q, QF, VEC, false, RC>(
        C, ldc, py, pscale, n, i0, i1,
        [&](int i) {
            stage_rows<RC>(i, i1, M, rM, S, rS, a, rA, z, rZ);
            stage_rows<RC>(i, i1, er_row, rE, zg_row, rG, nullptr, nullptr);
        },
        [&](int i, int slot, const auto *cst) {
        const double Mi = rM[slot], ai = rA[slot], zi = rZ[slot], aS = ai / rS[slot];
        const double es = rE[slot] * inv_er1;   // rank-one factor e_r,i / ||e_r||_1
        const double zg = rG[slot];
        const double lr = log_tab(ai, ltab) - log_tab(rS[slot], ltab);   // per row, all threads
        // A thread's columns are the same in every row, so the compiler would hoist their
        // loads out of the row loop and spill them at this register budget.  The pointers
        // are made opaque per row to keep the loads in the loop; e_c of entry e + 1 is loaded
        // while entry e is computed, y and gamma only where X_ij > 0.
        const double *yv = y, *ecv = ec, *gv = gamma;
        asm volatile("" : "+s"(yv), "+s"(ecv), "+s"(gv));
        int jn = slot_col<QF, NT, VEC>(0, n);
        double nec = ecv[jn];
        // this row: sum of e_c,j x_ij where X_ij = 0; e_c and e_c log e_c where X_ij > 0
        double u_ecxa = 0.0, x_ec = 0.0, x_lec = 0.0;
#pragma unroll 2
        for (int e = 0; e < E; ++e) {
            const bool valid = slot_valid<QF, NT, VEC>(e, n);
            const int j = jn;
            const double ecj = nec;
            if (e + 1 < E) {
                jn = slot_col<QF, NT, VEC>(e + 1, n);
                nec = ecv[jn];
            }
            const double c = valid ? (double)cst[e] : 0.0;
            const double xa = valid ? add_lo<LO>(fma(-sigma, c, wl[j] - Mi), wl, n, j) : -INFINITY;
            const double Xv = exp_tab_z(xa, etab) * aS;
            t_cf = fma(c, c, t_cf);
            if (Xv > 0.0) {
                // X_ij > 0 (valid): the full term
                const double f = (zi * Xv) * yv[j];
                const double xh = fma(es, ecj, f);   // >= f > 0
                const double lx = lr + xa;
                const double lxh = log_tab(xh, ltab);
                t_dphi += (xh * (lxh - lx) - xh) + Xv;
                t_cxh = fma(c, xh, t_cxh);
                t_cx = fma(c, Xv, t_cx);
                t_xhmin = fmin(t_xhmin, xh);
                t_xu = fma(Xv, (c - gv[j]) - zg, t_xu);
                t_xf = fma(Xv, Xv, t_xf);
                x_ec += ecj;
                x_lec += ecj > 0.0 ? ecj * log_tab(ecj, ltab) : 0.0;
                if (xhat)
                    xhat[(int64_t)i * ldx + col_of<NT, VEC>(e)] = xh;
            } else if (valid) {
                // X_ij = 0: Xhat_ij = es e_c,j, whose term es e_c,j (log es + log e_c,j - lr -
                // x_ij - 1) is added once per row below
                const double xr = es * ecj;
                u_ecxa = fma(ecj, xa, u_ecxa);
                t_cxh = fma(c, xr, t_cxh);
                t_xhmin = fmin(t_xhmin, xr);
                if (xhat)
                    xhat[(int64_t)i * ldx + col_of<NT, VEC>(e)] = xr;
            }
        }
        if (es > 0.0)
            t_dphi += es * ((log_tab(es, ltab) - lr - 1.0) * (t_sec - x_ec) + (t_slec - x_lec) -
                            u_ecxa);
        });
    double fin[7] = {t_dphi, t_cxh, t_cx, t_xu, t_xhmin, t_xf, t_cf};
    RedEnd::run_once(fin, lds);
    if (threadIdx.x == 0) {
        double *o = rowpart + (int64_t)blockIdx.x * STOP2_NSLOT;
        o[STOP2_DPHI] = fin[0];
        o[STOP2_CXH] = fin[1];
        o[STOP2_CX] = fin[2];
        o[STOP2_XU] = fin[3];
        o[STOP2_XHMIN] = fin[4];
        o[STOP2_XF] = fin[5];
        o[STOP2_CF] = fin[6];
        o[STOP2_NEG] = 0.0;
    }
}

// ---------------------------------------------------------------------------------
// column reduction: out_j = sum_g part[g][j], g ascending within each of NW strided
// subsets, subsets added in order.  64 columns per workgroup.
// ---------------------------------------------------------------------------------
template <int NW>
__global__ __launch_bounds__(NW *WAVE) void k_colreduce(const double *__restrict__ part, int G, int n,
                                                        double *__restrict__ out,
                                                        const double *__restrict__ sub,
                                                        double *__restrict__ out2)
{
    __shared__ double s[NW][WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int j = blockIdx.x * WAVE + lane;
    double acc = 0.0;
    if (j < n) {
#pragma unroll 8   // independent loads in flight; the additions keep their order
        for (int g = wv; g < G; g += NW)
            acc += part[(int64_t)g * n + j];
    }
    s[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && j < n) {
        double t = s[0][lane];
        for (int k = 1; k < NW; ++k)
            t += s[k][lane];
        out[j] = t;
        if (sub)
            out2[j] = t - sub[j];
    }
}

}  // namespace

// Tiles (NT threads, Q vector slots per thread, QF slabs always inside the row).  Each
// tile serves n in (previous capacity, NT*Q*VEC], so the first QF slabs are full for
// every n it is chosen for.  Light tiles serve eval and both stop passes (stop pass 2 is
// split into 2a and 2b so that neither holds a row's values across a reduction; its
// static LDS, with 8- and 32-row chunks of row scalars, is sized for the light tile); the
// heavy tile of the same row serves trial and sparsify, which keep more values live per
// entry; both run on the same grid.  1024-thread tiles keep 10 entries per thread at
// n <= 10240 (FP64), which leaves room for four waves per SIMD.  This table is the default;
// ibsn_autotune times the other compiled tiles that hold the row (tile_candidates) and
// grids of 1, 2 and 4 workgroups per CU on a problem, and records its choice per shape.
struct TileRow {
    int cap;                  // largest n served
    int nt, q, qf;            // light tile
    int nt_h, q_h, qf_h;      // heavy tile
    int per_cu;               // workgroups per CU
};
const TileRow TILES64[] = {
    {512, 256, 1, 0, 256, 1, 0, 4},      {1024, 256, 2, 1, 256, 2, 1, 4},
    {1536, 256, 3, 2, 256, 3, 2, 4},     {2048, 256, 4, 3, 256, 4, 3, 4},
    {3072, 512, 3, 2, 512, 3, 2, 2},     {4096, 512, 4, 3, 512, 4, 3, 2},
    {6144, 1024, 3, 2, 512, 6, 4, 1},    {8192, 1024, 4, 3, 512, 8, 6, 1},
    {10240, 1024, 5, 4, 512, 10, 8, 1},
};
const TileRow TILES32[] = {
    {1024, 256, 1, 0, 256, 1, 0, 4},     {2048, 256, 2, 1, 256, 2, 1, 4},
    {3072, 256, 3, 2, 256, 3, 2, 4},     {4096, 256, 4, 3, 256, 4, 3, 4},
    {6144, 512, 3, 2, 512, 3, 2, 2},     {8192, 512, 4, 3, 512, 4, 3, 2},
    {12288, 1024, 3, 2, 512, 6, 4, 1},   {16384, 1024, 4, 3, 512, 8, 6, 1},
    {20480, 512, 10, 8, 512, 10, 8, 1},
};
bool plan_rows(int64_t m, int64_t n, int cost_kind, int num_cus, RowPlan *p)
{
    const TileRow *t = cost_kind == 1 ? TILES32 : TILES64;
    const int nt = (int)(sizeof(TILES64) / sizeof(TILES64[0]));
    for (int k = 0; k < nt; ++k) {
        if (n <= t[k].cap) {
            p->nt = t[k].nt;
            p->q = t[k].q;
            p->qf = t[k].qf;
            p->nt_h = t[k].nt_h;
            p->q_h = t[k].q_h;
            p->qf_h = t[k].qf_h;
            p->vec = cost_kind == 1 ? 4 : 2;
            const int64_t g = (int64_t)num_cus * t[k].per_cu;
            p->grid = (int)(g < m ? g : m);
            p->nb = 1;
            p->bw = n;
            return true;
        }
    }
    return false;
}

int tile_candidates(int64_t n, int cost_kind, bool heavy, int (*out)[3], int cap)
{
    const int vec = cost_kind == 1 ? 4 : 2;
    int cnt = 0;
#define X(NT_, Q_, QF_)                                                                    \
    if (cnt < cap && (int64_t)NT_ * Q_ * vec >= n && (int64_t)NT_ * QF_ * vec <= n) {      \
        out[cnt][0] = NT_;                                                                 \
        out[cnt][1] = Q_;                                                                  \
        out[cnt][2] = QF_;                                                                 \
        ++cnt;                                                                             \
    }
    if (heavy) {
        IBSN_HEAVY_TILES(X)
    } else {
        IBSN_LIGHT_TILES(X)
    }
#undef X
    return cnt;
}

RowPlan heavy_plan(const RowPlan &p)
{
    RowPlan h = p;
    h.nt = p.nt_h;
    h.q = p.q_h;
    h.qf = p.qf_h;
    return h;
}

hipError_t launch_stop1(const RowPlan &p, const DenseArgs &d, const double *M, const double *S,
                        double *z, double *colpart, double *colpart2, double *rowpart,
                        hipStream_t st, double *rsum, const double *zin)
{
#define BODY                                                                                     \
    static LdsCache lc_, lcs_; \
    const size_t lds_bytes = lds_w2(d.n, lo_tile(NT, Q, VEC)); \
    if (rsum || zin) { \
        if (hipError_t e_ = lds_check((const void *)k_stop1<NT, Q, QF, VEC, CT, true>, lds_bytes, lcs_); e_ != hipSuccess) \
            return e_; \
        hipLaunchKernelGGL((k_stop1<NT, Q, QF, VEC, CT, true>), dim3(p.grid), dim3(NT), lds_bytes, st, \
                           (const CT *)d.C, d.ldc, d.py, d.pscale, (int)d.m, (int)d.n, d.sigma, d.w, \
                           d.wlo, d.a, M, S, z, colpart, colpart2, rowpart, rsum, zin); \
        return hipGetLastError(); \
    } \
    if (hipError_t e_ = lds_check((const void *)k_stop1<NT, Q, QF, VEC, CT, false>, lds_bytes, lc_); e_ != hipSuccess) \
        return e_; \
    hipLaunchKernelGGL((k_stop1<NT, Q, QF, VEC, CT, false>), dim3(p.grid), dim3(NT), lds_bytes, st,                 \
                       (const CT *)d.C, d.ldc, d.py, d.pscale, (int)d.m, (int)d.n, d.sigma, d.w, d.wlo, d.a, M, S, z,   \
                       colpart, colpart2, rowpart, rsum, zin)
#define X(a, b, c) IBSN_DISPATCH(a, b, c, BODY)
    IBSN_LIGHT_TILES(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

hipError_t launch_stop2(const RowPlan &p, const DenseArgs &d, const double *M, const double *S,
                        const Stop2Vec &v, double *xhat, double *rowpart, hipStream_t st,
                        int which, double *rowred)
{
#define BODY                                                                                      \
    static LdsCache lca_, lcb_;                                                                   \
    const size_t lds_bytes = lds_w2(d.n, lo_tile(NT, Q, VEC));                                    \
    if (hipError_t e_ = lds_check((const void *)k_stop2a<NT, Q, QF, VEC, CT>, lds_bytes, lca_);   \
        e_ != hipSuccess)                                                                         \
        return e_;                                                                                \
    if (hipError_t e_ = lds_check((const void *)k_stop2b<NT, Q, QF, VEC, CT>, lds_bytes, lcb_);   \
        e_ != hipSuccess)                                                                         \
        return e_;                                                                                \
    if (which & 1)                                                                                \
        hipLaunchKernelGGL((k_stop2a<NT, Q, QF, VEC, CT>), dim3(p.grid), dim3(NT), lds_bytes, st, \
                           (const CT *)d.C, d.ldc, d.py, d.pscale, (int)d.m, (int)d.n, d.sigma, d.w, \
                           d.wlo, d.a, M, S, v.gamma, v.psi, v.y, v.z, v.er_row, v.zg_row, rowpart, \
                           rowred);                                                               \
    if (which & 2)                                                                                \
        hipLaunchKernelGGL((k_stop2b<NT, Q, QF, VEC, CT>), dim3(p.grid), dim3(NT), lds_bytes, st, \
                           (const CT *)d.C, d.ldc, d.py, d.pscale, (int)d.m, (int)d.n, d.sigma, d.w, \
                           d.wlo, d.a, M, S, v.gamma, v.y, v.ec, v.z, v.er_row, v.zg_row, v.er1,  \
                           xhat, rowpart, d.ldo)
#define X(a, b, c) IBSN_DISPATCH(a, b, c, BODY)
    IBSN_LIGHT_TILES(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

hipError_t launch_colreduce(const double *part, int G, int64_t n, double *out, const double *sub,
                            double *out2, hipStream_t st)
{
    const int blocks = (int)((n + WAVE - 1) / WAVE);
    hipLaunchKernelGGL((k_colreduce<16>), dim3(blocks), dim3(16 * WAVE), 0, st, part, G, (int)n,
                       out, sub, out2);
    return hipGetLastError();
}

}  // namespace ibsn
