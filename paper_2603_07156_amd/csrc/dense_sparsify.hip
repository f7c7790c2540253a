// dense_sparsify.hip -- the sparsification pass (Algorithm 1) on gfx950; helpers in dense_common.h.
#include "dense_common.h"

namespace ibsn {
namespace {

// ---------------------------------------------------------------------------------
// Algorithm 1.  p = exp(theta - M_i)/S_i; rows i != istar keep p >= rho and divide
// by the kept sum; row istar is kept whole.  Compaction: per (slab q, wave) a ballot
// per vector lane gives the wave's kept count and each lane's rank; an exclusive scan of
// the counts of all (q, wave) segments, in column order, gives each segment's base.
// Entries go to the row's slot [i*n, i*n + len_i) in ascending column order.
// MX (mixed precision): p from the FP32 exponential (the threshold test is taken on that
// value, widened), kept values stored as FP32; sums stay FP64, and d = P~^T (a o P~ 1) for
// the stored factor P~.
// Column block of a split row (SPLIT): the block's kept entries go to the row's slot from
// column coff on (row pitch ldo), unnormalised, with the block's kept sum in ksum and its
// count in len, and no column partials; the row's blocks are joined and normalised
// afterwards.
// ---------------------------------------------------------------------------------
template <int NT, int Q, int QF, int VEC, typename CT, bool MX, bool SPLIT>
__global__ __launch_bounds__(NT) void k_sparsify(const CT *__restrict__ C, int64_t ldc,
                                              const double *__restrict__ py, double pscale, int m, int n,
                                                 double sigma, const double *__restrict__ w,
                                                 const double *__restrict__ wlo,
                                                 const double *__restrict__ a,
                                                 const double *__restrict__ M,
                                                 const double *__restrict__ S, double rho,
                                                 const int *__restrict__ istar_p,
                                                 int32_t *__restrict__ col,
                                                 xval_t<MX> *__restrict__ val,
                                                 int32_t *__restrict__ len,
                                                 double *__restrict__ colpart, int64_t ldo,
                                                 int coff, double *__restrict__ ksum)
{
    constexpr int E = Q * VEC;
    constexpr int NW = NT / WAVE;
    constexpr bool LO = lo_tile(NT, Q, VEC);
    using RedSum = BlockRed<NT, OP_SUM>;
    __shared__ double lds[RedSum::LDS];
    __shared__ int cnt[2][Q * NW];
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    extern __shared__ double wl[];   // w staged in LDS (n doubles, then the FP32 low parts)
    __shared__ double etab[EXP_TAB];
    __shared__ double rM[ROWCH], rS[ROWCH], rA[ROWCH];
    double acc[E];
    xval_t<MX> x[E];
    const int istar = *istar_p;
    exp_table_init(etab);
    stage_w2<LO>(w, wlo, n, wl);
#pragma unroll
    for (int e = 0; e < E; ++e)
        acc[e] = 0.0;
    row_loop<NT, Q, QF, VEC>(
        C, ldc, py, pscale, n, i0, i1, [&](int i) { stage_rows(i, i1, M, rM, S, rS, a, rA); },
        [&](int i, int slot, const auto *xr) {
        const double Mi = rM[slot], iS = 1.0 / rS[slot];
        // an index offset the compiler cannot see through keeps the row-invariant LDS reads
        // of w in the row loop (hoisted, they spill at this register budget)
        int zo = 0;
        asm volatile("" : "+v"(zo));
        const bool dense = (i == istar);
        int *cn = cnt[i & 1];
        double red[1] = {0.0};
        unsigned long long keepbits = 0;
        // per slab: this lane's rank among the wave's kept entries (lanes below, all
        // vector slots) and the wave's kept count
        int rank[Q], wcnt[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            rank[q] = 0;
            wcnt[q] = 0;
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool valid = slot_valid<QF, NT, VEC>(e, n);
            const int j = slot_col<QF, NT, VEC>(e, n) + zo;
            const double xa = add_lo<LO>(fma(-sigma, (double)xr[e], wl[j] - Mi), wl, n, j);
            const double p = exp_pass_z<MX>(valid ? xa : -INFINITY, etab) * iS;
            const bool keep = valid && (dense || p >= rho);
            x[e] = (xval_t<MX>)p;
            if (keep) {
                keepbits |= 1ull << e;
                red[0] += p;
            }
            const unsigned long long bal = __ballot(keep);
            rank[e / VEC] += __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
            wcnt[e / VEC] += __popcll(bal);
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
                cn[q * NW + wv] = wcnt[q];
        }
        RedSum::run(red, lds, parity);   // its barrier also publishes cn[]
        const double ik = 1.0 / red[0];   // 1 / kept row sum
        // exclusive scan of the Q*NW segment counts (column order), 64 per wave scan
        constexpr int NSEG = Q * NW, NCH = (NSEG + WAVE - 1) / WAVE;
        int running = 0, base[Q];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int f = c * WAVE + lane;
            const int v = f < NSEG ? cn[f] : 0;
            const int inc = wave_scan_incl(v) + running;
            const int exc = inc - v;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int fq = q * NW + wv;   // the same in all lanes of the wave
                const int b = __builtin_amdgcn_ds_bpermute((fq & (WAVE - 1)) * 4, exc);
                if (fq / WAVE == c)
                    base[q] = b;
            }
            running = __builtin_amdgcn_ds_bpermute((WAVE - 1) * 4, inc);
        }
        const double ai = rA[slot];
        double rs = 0.0;   // MX: sum of the row's stored values
        const int64_t rbase = SPLIT ? (int64_t)i * ldo + coff : (int64_t)i * n;
        int32_t *crow = col + rbase;
        xval_t<MX> *vrow = val + rbase;
        const bool asis = SPLIT || dense;   // stored without the division by the kept sum
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            int before = rank[q];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const int e = q * VEC + v;
                if (keepbits & (1ull << e)) {
                    // d = P_rho^T a from the values as stored, so that H_rho 1 = 0 holds
                    // for the factor the HVP reads
                    const xval_t<MX> pv =
                        (xval_t<MX>)(asis ? (double)x[e] : (double)x[e] * ik);
                    const int pos = base[q] + before;
                    crow[pos] = col_of<NT, VEC>(e) + (SPLIT ? coff : 0);
                    vrow[pos] = pv;
                    if constexpr (MX) {
                        x[e] = pv;
                        rs += (double)pv;
                    } else {
                        acc[e] = fma(ai, (double)pv, acc[e]);
                    }
                    ++before;
                }
            }
        }
        if (MX && !SPLIT) {
            // FP32 values make the stored row sum 1 + O(2^-24) rather than 1; with
            // d = P~^T (a o P~ 1) the stored factor P~ still gives H_rho 1 = 0 and a
            // positive semidefinite H_rho (Theorem 3.2)
            double t[1] = {rs};
            RedSum::run(t, lds, parity);
            const double sc = ai * t[0];
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (keepbits & (1ull << e))
                    acc[e] = fma(sc, (double)x[e], acc[e]);
        }
        if (threadIdx.x == 0) {
            len[i] = running;
            if (SPLIT)
                ksum[i] = red[0];
        }
        });
    if (!SPLIT)
        store_cols<NT, Q, VEC>(colpart + (int64_t)blockIdx.x * n, n, acc);
}

}  // namespace

hipError_t launch_sparsify(const RowPlan &p_in, const DenseArgs &d, const double *M, const double *S,
                           double rho, const int *istar, int32_t *col, void *val, int32_t *len,
                           double *colpart, hipStream_t st, double *ksum)
{
    const RowPlan p = heavy_plan(p_in);
#define BODY                                                                                     \
    static LdsCache lc_, lcs_; \
    const size_t lds_bytes = lds_w2(d.n, lo_tile(NT, Q, VEC)); \
    if (ksum) { \
        if (hipError_t e_ = lds_check((const void *)k_sparsify<NT, Q, QF, VEC, CT, MX, true>, lds_bytes, lcs_); e_ != hipSuccess) \
            return e_; \
        hipLaunchKernelGGL((k_sparsify<NT, Q, QF, VEC, CT, MX, true>), dim3(p.grid), dim3(NT), lds_bytes, st, \
                           (const CT *)d.C, d.ldc, d.py, d.pscale, (int)d.m, (int)d.n, d.sigma, d.w, \
                           d.wlo, d.a, M, S, rho, istar, col, (xval_t<MX> *)val, len, colpart, d.ldo, \
                           (int)d.coff, ksum); \
        return hipGetLastError(); \
    } \
    if (hipError_t e_ = lds_check((const void *)k_sparsify<NT, Q, QF, VEC, CT, MX, false>, lds_bytes, lc_); e_ != hipSuccess) \
        return e_; \
    hipLaunchKernelGGL((k_sparsify<NT, Q, QF, VEC, CT, MX, false>), dim3(p.grid), dim3(NT), lds_bytes, st, \
                       (const CT *)d.C, d.ldc, d.py, d.pscale, (int)d.m, (int)d.n, d.sigma, d.w, d.wlo, d.a, M, S, rho, \
                       istar, col, (xval_t<MX> *)val, len, colpart, d.ldo, (int)d.coff, ksum)
#define X(a, b, c) IBSN_DISPATCH_MX(a, b, c, BODY)
    IBSN_HEAVY_TILES(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

}  // namespace ibsn
