// dense_sparsify.hip -- the sparsification pass (Algorithm 1) on gfx950; helpers in dense_common.h.
#include "dense_common.h"

namespace ibsn {
namespace {

// ---------------------------------------------------------------------------------
// Algorithm 1.  p = exp(theta - M_i)/S_i; rows i != istar keep p >= rho and divide
// by the kept sum; row istar is kept whole.  Compaction: per (slab q, wave) a ballot
// per vector lane gives the wave's kept count and each lane's rank; the counts of all
// (q, wave) segments, in column order, give each segment's base.  Entries go to the
// row's slot [i*n, i*n + len_i) in ascending column order.
// ---------------------------------------------------------------------------------
template <int NT, int Q, int QF, int VEC, typename CT>
__global__ __launch_bounds__(NT) void k_sparsify(const CT *__restrict__ C, int64_t ldc, int m, int n,
                                                 double sigma, const double *__restrict__ w,
                                                 const double *__restrict__ a,
                                                 const double *__restrict__ M,
                                                 const double *__restrict__ S, double rho,
                                                 const int *__restrict__ istar_p,
                                                 int32_t *__restrict__ col,
                                                 double *__restrict__ val,
                                                 int32_t *__restrict__ len,
                                                 double *__restrict__ colpart)
{
    constexpr int E = Q * VEC;
    constexpr int NW = NT / WAVE;
    using RedSum = BlockRed<NT, OP_SUM>;
    __shared__ double lds[RedSum::LDS];
    __shared__ int cnt[2][Q * NW];
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const unsigned long long lt = (1ull << lane) - 1ull;
    extern __shared__ double wl[];   // w staged in LDS (n doubles)
    __shared__ double etab[EXP_TAB];
    __shared__ double rM[ROWCH], rS[ROWCH], rA[ROWCH];
    double acc[E], x[E];
    const int istar = *istar_p;
    exp_table_init(etab);
    stage_lds(w, n, wl);
#pragma unroll
    for (int e = 0; e < E; ++e)
        acc[e] = 0.0;
    row_loop<NT, Q, QF, VEC>(
        C, ldc, n, i0, i1, [&](int i) { stage_rows(i, i1, M, rM, S, rS, a, rA); },
        [&](int i, int slot, const CT *xr) {
        const double Mi = rM[slot], iS = 1.0 / rS[slot];
        const bool dense = (i == istar);
        int *cn = cnt[i & 1];
        double red[1] = {0.0};
        unsigned long long keepbits = 0;
        unsigned long long bal[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = col_of<NT, VEC>(e);
            const bool valid = slot_valid<QF, NT, VEC>(e, n);
            const double xa = fma(-sigma, (double)xr[e], wl[slot_col<QF, NT, VEC>(e, n)] - Mi);
            const double p = exp_tab(valid ? xa : -INFINITY, etab) * iS;
            const bool keep = valid && (dense || p >= rho);
            x[e] = p;
            if (keep) {
                keepbits |= 1ull << e;
                red[0] += p;
            }
            bal[e] = __ballot(keep);
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                int c = 0;
#pragma unroll
                for (int v = 0; v < VEC; ++v)
                    c += __popcll(bal[q * VEC + v]);
                cn[q * NW + wv] = c;
            }
        }
        RedSum::run(red, lds, parity);   // its barrier also publishes cn[]
        const double ik = 1.0 / red[0];   // 1 / kept row sum
        int running = 0, base[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            for (int k = 0; k < NW; ++k) {
                if (k == wv)
                    base[q] = running;
                running += cn[q * NW + k];
            }
        }
        const double ai = rA[slot];
        int32_t *crow = col + (int64_t)i * n;
        double *vrow = val + (int64_t)i * n;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            int before = 0;
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                before += __popcll(bal[q * VEC + v] & lt);
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const int e = q * VEC + v;
                if (keepbits & (1ull << e)) {
                    const double pv = dense ? x[e] : x[e] * ik;
                    const int pos = base[q] + before;
                    crow[pos] = col_of<NT, VEC>(e);
                    vrow[pos] = pv;
                    acc[e] = fma(ai, pv, acc[e]);
                    ++before;
                }
            }
        }
        if (threadIdx.x == 0)
            len[i] = running;
        });
    store_cols<NT, Q, VEC>(colpart + (int64_t)blockIdx.x * n, n, acc);
}

}  // namespace

hipError_t launch_sparsify(const RowPlan &p_in, const DenseArgs &d, const double *M, const double *S,
                           double rho, const int *istar, int32_t *col, double *val, int32_t *len,
                           double *colpart, hipStream_t st)
{
    const RowPlan p = heavy_plan(p_in);
    const size_t lds_bytes = (size_t)d.n * sizeof(double);
#define BODY                                                                                     \
    hipLaunchKernelGGL((k_sparsify<NT, Q, QF, VEC, CT>), dim3(p.grid), dim3(NT), lds_bytes, st,              \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.w, d.a, M, S, rho, \
                       istar, col, val, len, colpart)
#define X(a, b, c) IBSN_DISPATCH(a, b, c, BODY)
    IBSN_HEAVY_TILES(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

}  // namespace ibsn
