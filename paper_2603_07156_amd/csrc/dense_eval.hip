// dense_eval.hip -- the subproblem eval (row LSE) pass on gfx950; helpers in dense_common.h.
#include "dense_common.h"

namespace ibsn {
namespace {

// ---------------------------------------------------------------------------------
// eval: M_i = max_j theta_ij, S_i = sum_j exp(theta_ij - M_i), column partials of
// a_i P_ij, objective row terms a_i ((r_i + M_i) + log S_i).
// MX (mixed precision): exp(theta_ij - m_w) in FP32 and held as FP32; the argument, the
// shifts, S_i, the column partials and the objective stay FP64.
// Column block of a split row (SPLIT): the first launch per block (colpart null) writes the
// block's M and S; the second (Mfull given) takes the row's combined shift Mfull_i and the
// factor f_i = a_i / S_i of the whole row, so that its column partials and plan entries
// (row pitch ldp) are f_i exp(theta_ij - Mfull_i) = a_i P_ij; it writes no row outputs.
// ---------------------------------------------------------------------------------
template <int NT, int Q, int QF, int VEC, typename CT, bool MX, bool SPLIT>
__global__ __launch_bounds__(NT) void k_eval(const CT *__restrict__ C, int64_t ldc,
                                              const double *__restrict__ py, double pscale, int m, int n,
                                             double sigma, double qg,
                                             const double *__restrict__ w,
                                             const double *__restrict__ wlo,
                                             const double *__restrict__ a,
                                             const double *__restrict__ r, double *__restrict__ Mo,
                                             double *__restrict__ So, double *__restrict__ lse,
                                             double *__restrict__ plan,
                                             double *__restrict__ colpart,
                                             double *__restrict__ rowpart, int64_t ldp,
                                             const double *__restrict__ Mfull,
                                             const double *__restrict__ fscale)
{
    constexpr int E = Q * VEC;
    constexpr int NW = NT / WAVE;
    constexpr bool LO = lo_tile(NT, Q, VEC);
    // per row: each wave takes its own shift m_w = grid(wave max of theta) and sums
    // exp(theta - m_w); one barrier publishes the (m_w, s_w) pairs; every wave then forms
    // M = max_w m_w = grid(max theta) (grid rounding is monotone) and
    // S = sum_w s_w exp(m_w - M), and scales its entries by exp(m_w - M).  All shifts
    // lie on the grid, so m_w - M is exact.  The pair buffer alternates between rows.
    __shared__ double pairs[2][2 * NW];
    __shared__ double etab[EXP_TAB];
    // log S_i for the row outputs, by thread 0: the table log keeps wave 0 from falling
    // ~75 instructions (the library log) behind the other waves at every row's barrier
    __shared__ __align__(16) double ltab[2 * LOG_TAB];
    extern __shared__ double wl[];   // w staged in LDS (n doubles, then the FP32 low parts)
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    log_table_init(ltab);
    exp_table_init(etab);   // its barrier also publishes ltab
    stage_w2<LO>(w, wlo, n, wl);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    __shared__ double rA[ROWCH], rR[ROWCH];
    double acc[E];
    xval_t<MX> x[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        acc[e] = 0.0;
    double rowacc = 0.0;
    row_loop<NT, Q, QF, VEC>(
        C, ldc, py, pscale, n, i0, i1,
        [&](int i) {
            if (SPLIT && Mfull)
                stage_rows(i, i1, fscale, rA, Mfull, rR, nullptr, nullptr);
            else
                stage_rows(i, i1, a, rA, r, rR, nullptr, nullptr);
        },
        [&](int i, int slot, const auto *xr) {
        // padding slots: theta = -inf, so they drop out of the max and p = 0; a wave
        // with no column in the row gets m_w = -inf, s_w = 0 and factor 0.  The shift is
        // taken from the high parts alone (any value near the maximum serves).
        double mt = -INFINITY;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double th = fma(-sigma, (double)xr[e], wl[slot_col<QF, NT, VEC>(e, n)]);
            mt = fmax(mt, slot_valid<QF, NT, VEC>(e, n) ? th : -INFINITY);
        }
        const double mw = grid(wave_red<OP_MAX>(mt), qg);
        double st = 0.0;
        // the low parts are the same in every row: an index offset the compiler cannot
        // see through keeps their LDS reads in the row loop (hoisted, they spill)
        int zo = 0;
        asm volatile("" : "+v"(zo));
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = slot_col<QF, NT, VEC>(e, n);
            const double xa =
                add_lo<LO>(fma(-sigma, (double)xr[e], wl[j] - mw), wl, n, j + zo);
            const double p =
                exp_pass_z<MX>(slot_valid<QF, NT, VEC>(e, n) ? xa : -INFINITY, etab);
            x[e] = (xval_t<MX>)p;   // exact: in the mixed form p is already an FP32 value
            st += p;
        }
        const double sw = wave_red<OP_SUM>(st);
        double *pr = pairs[parity];
        parity ^= 1;
        if (lane == 0) {
            pr[wv] = mw;
            pr[NW + wv] = sw;
        }
        __syncthreads();
        static_assert(NW <= 16, "the wave pairs are combined within one row of lanes");
        const double mk = lane < NW ? pr[lane] : -INFINITY;
        const double M = row0_red<OP_MAX>(mk);
        const double term = lane < NW ? pr[NW + lane] * exp_tab(mk - M, etab) : 0.0;
        const double S = row0_red<OP_SUM>(term);
        const double ai = rA[slot];
        // a_i exp(m_w - M) / S, or f_i exp(m_w - Mfull_i) for the second launch of a block
        const double sc = (SPLIT && Mfull) ? ai * exp_tab(mw - rR[slot], etab)
                                           : ai / S * exp_tab(mw - M, etab);
#pragma unroll
        for (int e = 0; e < E; ++e)
            acc[e] = fma(sc, (double)x[e], acc[e]);
        if (plan) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = col_of<NT, VEC>(e);
                if (j < n)
                    plan[(int64_t)i * (SPLIT ? ldp : n) + j] = sc * (double)x[e];
            }
        }
        if (threadIdx.x == 0 && !(SPLIT && Mfull)) {
            const double ls = log_tab(S, ltab);
            Mo[i] = M;
            So[i] = S;
            if (lse)
                lse[i] = M + ls;
            if (r)
                rowacc += ai * ((rR[slot] + M) + ls);
        }
        });
    if (!SPLIT || colpart)
        store_cols<NT, Q, VEC>(colpart + (int64_t)blockIdx.x * n, n, acc);
    if (threadIdx.x == 0 && (!SPLIT || rowpart))
        rowpart[blockIdx.x] = rowacc;
}

}  // namespace

hipError_t launch_eval(const RowPlan &p, const DenseArgs &d, const double *r, double *M, double *S,
                       double *lse, double *plan, double *colpart, double *rowpart, hipStream_t st,
                       const double *Mfull, const double *fscale)
{
#define BODY                                                                                     \
    static LdsCache lc_, lcs_; \
    const size_t lds_ = lds_w2(d.n, lo_tile(NT, Q, VEC)); \
    if (Mfull || !colpart) { \
        if (hipError_t e_ = lds_check((const void *)k_eval<NT, Q, QF, VEC, CT, MX, true>, lds_, lcs_); e_ != hipSuccess) \
            return e_; \
        hipLaunchKernelGGL((k_eval<NT, Q, QF, VEC, CT, MX, true>), dim3(p.grid), dim3(NT), lds_, st, \
                           (const CT *)d.C, d.ldc, d.py, d.pscale, (int)d.m, (int)d.n, d.sigma, d.q, \
                           d.w, d.wlo, d.a, r, M, S, lse, plan, colpart, rowpart, d.ldo, Mfull, fscale); \
        return hipGetLastError(); \
    } \
    if (hipError_t e_ = lds_check((const void *)k_eval<NT, Q, QF, VEC, CT, MX, false>, lds_, lc_); e_ != hipSuccess) \
        return e_; \
    hipLaunchKernelGGL((k_eval<NT, Q, QF, VEC, CT, MX, false>), dim3(p.grid), dim3(NT),                     \
                       lds_, st,                                         \
                       (const CT *)d.C, d.ldc, d.py, d.pscale, (int)d.m, (int)d.n, d.sigma, d.q, d.w, d.wlo, d.a, r, M, S, \
                       lse,                                                                      \
                       plan, colpart, rowpart, d.ldo, Mfull, fscale)
#define X(a, b, c) IBSN_DISPATCH_MX(a, b, c, BODY)
    IBSN_LIGHT_TILES(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

}  // namespace ibsn
