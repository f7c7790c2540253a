// dense_trial.hip -- the Armijo trial pass on gfx950; helpers in dense_common.h.
#include "dense_common.h"

namespace ibsn {
namespace {

// ---------------------------------------------------------------------------------
// Armijo trial from the row state M of the base point, tau = t*Delta/eta:
//   q = exp(theta - M_i), A = sum q, small step (BIG=0, cv = expm1(tau)):
//   B = sum q*cv, qe = q + q*cv = q e^tau, delta = log1p(B/A);
//   big step (BIG=1, cv = exp(tau - tau_shift)): qe = q*cv, delta = tau_shift + log(Z/A).
//   Z = sum qe, P'_ij = qe / Z, new state M' = M + tau_shift + log(max qe), S' = Z / max qe.
// MX (mixed precision): q from the FP32 exponential and qe held as FP32; cv, the sums
// A, B, Z, the decrease and the new row state stay FP64.  The mixed form only takes steps
// with max tau <= 80 (q e^tau <= e^80 < FLT_MAX); larger steps go to the FP64 pass.
// `flags` selects the steps a launch handles: bit f for scal[SC_BIG] == f (0: max tau <=
// 80, 2: 80 < max tau <= 500, 1: larger, the shifted form).
// Column block of a split row: the first launch per block writes the row sums Z, A, B and
// the maximum of q e^tau over the block to rowred (four arrays of m) instead of the row
// outputs; the second (fscale given) takes f_i = a_i / Z_i of the whole row for its column
// partials and writes no row outputs.
// ---------------------------------------------------------------------------------
template <int NT, int Q, int QF, int VEC, typename CT, bool MX, int BIG, bool SPLIT>
__global__ __launch_bounds__(NT) void k_trial(const CT *__restrict__ C, int64_t ldc,
                                              const double *__restrict__ py, double pscale, int m, int n,
                                              double sigma, double qg,
                                              const double *__restrict__ w,
                                              const double *__restrict__ wlo,
                                              const double *__restrict__ a,
                                              const double *__restrict__ Mb,
                                              const double *__restrict__ colv,
                                              const double *__restrict__ scal,
                                              double *__restrict__ Mn, double *__restrict__ Sn,
                                              double *__restrict__ colpart,
                                              double *__restrict__ rowpart, int flags,
                                              double *__restrict__ rowred,
                                              const double *__restrict__ fscale)
{
    constexpr int E = Q * VEC;
    constexpr bool LO = lo_tile(NT, Q, VEC);
    using Red = BlockRed<NT, OP_SUM, OP_SUM, OP_SUM, OP_MAX>;
    __shared__ double lds[Red::LDS];
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    if (!((flags >> (int)scal[SC_BIG]) & 1))
        return;   // another launch of the trial handles this step
    const double tau_shift = scal[SC_TAUSHIFT];
    extern __shared__ double cvl[];   // colv staged in LDS (n doubles, then the low parts of w)
    __shared__ double etab[EXP_TAB];
    __shared__ double rM[ROWCH], rA[ROWCH];
    double wr[E], acc[E];
    xval_t<MX> x[E];
    exp_table_init(etab);
    load_w<NT, Q, VEC>(w, n, wr);   // padding slots: -inf, so q = 0 there
    stage_w2<LO>(colv, wlo, n, cvl);
#pragma unroll
    for (int e = 0; e < E; ++e)
        acc[e] = 0.0;
    double rowacc = 0.0;
    row_loop<NT, Q, QF, VEC>(
        C, ldc, py, pscale, n, i0, i1,
        [&](int i) {
            stage_rows(i, i1, Mb, rM, (SPLIT && fscale) ? fscale : a, rA, nullptr, nullptr);
        },
        [&](int i, int slot, const auto *xr) {
        const double Mi = rM[slot];
        // The staged column values are the same for every row; an index offset the compiler
        // cannot see through keeps their LDS reads in the row loop instead of hoisting them
        // into registers (which spills at this register budget).
        int zo = 0;
        asm volatile("" : "+v"(zo));
        // slot 0 (Z) is needed by every thread, the others by thread 0 only
        double red[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = slot_col<QF, NT, VEC>(e, n) + zo;
            const double q =
                exp_pass_z<MX>(add_lo<LO>(fma(-sigma, (double)xr[e], wr[e] - Mi), cvl, n, j), etab);
            const double cv = cvl[j];   // finite; q = 0 on padding
            red[1] += q;
            double qe;
            if constexpr (BIG) {
                qe = q * cv;
            } else {
                const double qf = q * cv;
                red[2] += qf;
                qe = q + qf;
            }
            red[0] += qe;
            red[3] = fmax(red[3], qe);
            x[e] = (xval_t<MX>)qe;
        }
        Red::template run_part<1>(red, lds, parity);
        const double Z = red[0], A = red[1], B = red[2], mx = red[3];
        const double ai = rA[slot];
        const double sc = (SPLIT && fscale) ? ai : ai / Z;
#pragma unroll
        for (int e = 0; e < E; ++e)
            acc[e] = fma(sc, (double)x[e], acc[e]);
        if (SPLIT && threadIdx.x == 0) {
            if (rowred) {
                rowred[i] = Z;
                rowred[m + i] = A;
                rowred[2 * (int64_t)m + i] = B;
                rowred[3 * (int64_t)m + i] = mx;
            }
        } else if (threadIdx.x == 0) {
            // a step that pushes a whole row below the FP64 range is not a decrease
            const double delta =
                !(Z > 0.0) ? INFINITY : (BIG ? tau_shift + log(Z / A) : log1p(B / A));
            rowacc += ai * delta;
            // new shift on the grid; S' carries the exact remainder so that
            // exp(x'_ij) / S'_i = P'_ij for the fresh x' of the point w + tau
            const double Mnew = grid(Mi + (tau_shift + log(mx)), qg);
            Mn[i] = Mnew;
            Sn[i] = Z * exp((Mi - Mnew) + tau_shift);
        }
        });
    if (!SPLIT || colpart)
        store_cols<NT, Q, VEC>(colpart + (int64_t)blockIdx.x * n, n, acc);
    if (!SPLIT && threadIdx.x == 0)
        rowpart[blockIdx.x] = rowacc;
}

}  // namespace

hipError_t launch_trial(const RowPlan &p_in, const DenseArgs &d, const double *M, const double *colv,
                        const double *scal, double *M_new, double *S_new, double *colpart,
                        double *rowpart, hipStream_t st, double *rowred, const double *fscale)
{
    const RowPlan p = heavy_plan(p_in);
    const bool split = rowred || fscale;
#define LAUNCH_TRIAL(MXV, BIGV, FLAGS, LC)                                                        \
    if (split) {                                                                                  \
        LAUNCH_TRIAL1(MXV, BIGV, FLAGS, LC##s, true);                                             \
    } else {                                                                                      \
        LAUNCH_TRIAL1(MXV, BIGV, FLAGS, LC, false);                                               \
    }
#define LAUNCH_TRIAL1(MXV, BIGV, FLAGS, LC, SPL)                                                  \
    if (hipError_t e_ = lds_check((const void *)k_trial<NT, Q, QF, VEC, CT, MXV, BIGV, SPL>,     \
                                  lds_w2(d.n, lo_tile(NT, Q, VEC)), LC);                          \
        e_ != hipSuccess)                                                                         \
        return e_;                                                                                \
    hipLaunchKernelGGL((k_trial<NT, Q, QF, VEC, CT, MXV, BIGV, SPL>), dim3(p.grid), dim3(NT),    \
                       lds_w2(d.n, lo_tile(NT, Q, VEC)), st,                                      \
                       (const CT *)d.C, d.ldc, d.py, d.pscale, (int)d.m, (int)d.n, d.sigma, d.q, d.w, \
                       d.wlo, d.a, M, colv, scal, M_new, S_new, colpart, rowpart, FLAGS, rowred, \
                       fscale)
    // FP64: the small form for flags 0 and 2, the shifted form for flag 1.  Mixed: the FP32
    // small form for flag 0 only; flags 2 and 1 run the FP64 forms.
#define BODY                                                                                      \
    static LdsCache lc0_, lc1_, lc2_, lc0_s, lc1_s, lc2_s;                                        \
    if constexpr (MX) {                                                                           \
        LAUNCH_TRIAL(true, 0, 1, lc2_);                                                           \
    }                                                                                             \
    LAUNCH_TRIAL(false, 0, MX ? 4 : 5, lc0_);                                                     \
    LAUNCH_TRIAL(false, 1, 2, lc1_)
#define X(a, b, c) IBSN_DISPATCH_MX(a, b, c, BODY)
    IBSN_HEAVY_TILES(X)
#undef X
#undef BODY
#undef LAUNCH_TRIAL
#undef LAUNCH_TRIAL1
    return hipErrorInvalidValue;
}

}  // namespace ibsn
