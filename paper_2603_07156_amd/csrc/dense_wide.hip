// dense_wide.hip -- rows wider than the register tiles, on gfx950.
//
// A row of more than one tile's width is split into nb column blocks of width bw (the last
// one narrower); every dense pass then runs its own kernel once per block, on the block's
// columns only (C, y, w and its low parts offset to the block's first column), and the
// kernels here join the blocks per row:
//   - eval: each block's shift M_b and sum S_b give the row's M = max_b M_b and
//     S = sum_b S_b exp(M_b - M) (all shifts on the grid, so M_b - M is exact); a second
//     launch per block forms the column partials a_i exp(theta_ij - M) / S from them.
//   - trial: the block sums Z, A, B and maxima of q e^tau add up (maximum) to the row's,
//     from which the decrease, the new row state and a_i / Z follow as in the one-block
//     kernel; a second launch per block forms the column partials.
//   - sparsify: each block writes its kept entries, unnormalised, at its own offset in the
//     row's slot, with its kept count and sum; the join moves the blocks' segments
//     together, divides by the row's kept sum (all but row i*) and forms the row weights of
//     d = P_rho^T a (a_i, or a_i times the stored row sum for FP32 values), and d is then
//     gathered column by column from the transpose.
//   - stop test: the blocks' row sums of X (pass 1) and of X y and the two minima
//     (pass 2a) join per row; pass 2b's sums are per workgroup and add up as they are.
// Per-block row arrays are nb consecutive m-vectors (block b at offset b m).  Each row is
// joined by one thread in block order, and per-row terms are summed per row range in a
// fixed order, so results are reproducible.
#include "dense_common.h"

namespace ibsn {
namespace {

constexpr int WNT = 256;

// rows [m g / G, m (g + 1) / G) of workgroup g
__device__ __forceinline__ void part_rows(int64_t m, int g, int G, int64_t &i0, int64_t &i1)
{
    i0 = m * g / G;
    i1 = m * (g + 1) / G;
}

// fixed-order sum of one value per thread (tree over the workgroup); result in thread 0
__device__ __forceinline__ double wsum(double v, double *lds)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = WNT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(WNT) void k_wide_eval_rows(int64_t m, int nb, int G,
                                                        const double *__restrict__ Mb,
                                                        const double *__restrict__ Sb,
                                                        const double *__restrict__ a,
                                                        const double *__restrict__ r,
                                                        double *__restrict__ M,
                                                        double *__restrict__ S,
                                                        double *__restrict__ lse,
                                                        double *__restrict__ f,
                                                        double *__restrict__ rowpart)
{
    __shared__ double lds[WNT];
    int64_t i0, i1;
    part_rows(m, blockIdx.x, G, i0, i1);
    double obj = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += WNT) {
        double Mi = -INFINITY;
        for (int b = 0; b < nb; ++b)
            Mi = fmax(Mi, Mb[b * m + i]);
        double Si = 0.0;
        for (int b = 0; b < nb; ++b)
            Si += Sb[b * m + i] * exp(Mb[b * m + i] - Mi);
        const double ls = log(Si);
        M[i] = Mi;
        S[i] = Si;
        f[i] = a[i] / Si;
        if (lse)
            lse[i] = Mi + ls;
        if (r)
            obj += a[i] * ((r[i] + Mi) + ls);
    }
    const double t = wsum(obj, lds);
    if (threadIdx.x == 0 && rowpart)
        rowpart[blockIdx.x] = t;
}

__global__ __launch_bounds__(WNT) void k_wide_trial_rows(int64_t m, int nb, int G,
                                                         const double *__restrict__ rr,
                                                         const double *__restrict__ a,
                                                         const double *__restrict__ Mb,
                                                         const double *__restrict__ scal,
                                                         double qg, double *__restrict__ Mn,
                                                         double *__restrict__ Sn,
                                                         double *__restrict__ f,
                                                         double *__restrict__ rowpart)
{
    __shared__ double lds[WNT];
    int64_t i0, i1;
    part_rows(m, blockIdx.x, G, i0, i1);
    const bool big = scal[SC_BIG] == 1.0;   // the shifted form ran
    const double tau_shift = scal[SC_TAUSHIFT];
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += WNT) {
        double Z = 0.0, A = 0.0, B = 0.0, mx = 0.0;
        for (int b = 0; b < nb; ++b) {
            const double *p = rr + 4 * m * b;
            Z += p[i];
            A += p[m + i];
            B += p[2 * m + i];
            mx = fmax(mx, p[3 * m + i]);
        }
        // a step that pushes a whole row below the FP64 range is not a decrease
        const double delta = !(Z > 0.0) ? INFINITY : (big ? tau_shift + log(Z / A) : log1p(B / A));
        acc += a[i] * delta;
        const double Mi = Mb[i];
        const double Mnew = grid(Mi + (tau_shift + log(mx)), qg);
        Mn[i] = Mnew;
        Sn[i] = Z * exp((Mi - Mnew) + tau_shift);
        f[i] = a[i] / Z;
    }
    const double t = wsum(acc, lds);
    if (threadIdx.x == 0)
        rowpart[blockIdx.x] = t;
}

// One wave per row: block b's kept entries move from column offset b bw of the row's slot
// to just after the blocks before it, each entry read and written once by the same lane
// (a left move, chunk by chunk in ascending order, so no entry is overwritten before it is
// read); rows other than istar are divided by their kept sum on the way.  col and val are
// not restrict: the moves read and write the same arrays.
template <typename VT>
__global__ __launch_bounds__(WAVE) void k_wide_join(int64_t m, int64_t n, int nb, int64_t bw,
                                                    const int32_t *__restrict__ lenb,
                                                    const double *__restrict__ ksb,
                                                    const double *__restrict__ a,
                                                    const int *__restrict__ istar_p,
                                                    int32_t *col, VT *val,
                                                    int32_t *__restrict__ len,
                                                    double *__restrict__ u)
{
    const int lane = threadIdx.x;
    const int istar = *istar_p;
    for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
        double ks = 0.0;
        for (int b = 0; b < nb; ++b)
            ks += ksb[b * m + i];
        const bool dense = (i == istar);
        const double ik = 1.0 / ks;
        int32_t *crow = col + i * n;
        VT *vrow = val + i * n;
        int64_t off = 0;
        double rs = 0.0;   // sum of the row's values as stored
        for (int b = 0; b < nb; ++b) {
            const int64_t src = b * bw, l = lenb[b * m + i];
            for (int64_t k = lane; k < l; k += WAVE) {
                const int32_t cj = crow[src + k];
                const VT v = vrow[src + k];
                const VT nv = dense ? v : (VT)((double)v * ik);
                crow[off + k] = cj;
                vrow[off + k] = nv;
                rs += (double)nv;
            }
            off += l;
        }
        rs = wave_red<OP_SUM>(rs);
        if (lane == 0) {
            len[i] = (int32_t)off;
            // d = P~^T (a o P~ 1) for FP32 values, P_rho^T a for FP64 (see k_sparsify)
            u[i] = sizeof(VT) == 4 ? a[i] * rs : a[i];
        }
    }
}

// d_j = sum over the transpose's column j (rows != istar, ascending) of u_i P_ij, plus the
// dense row istar's u P_istar,j
template <typename VT>
__global__ __launch_bounds__(WNT) void k_wide_d(int64_t n, const int64_t *__restrict__ colptr,
                                                const int32_t *__restrict__ rowidx,
                                                const VT *__restrict__ cval,
                                                const VT *__restrict__ val,
                                                const int *__restrict__ istar_p,
                                                const double *__restrict__ u,
                                                double *__restrict__ d)
{
    const int64_t j = (int64_t)blockIdx.x * WNT + threadIdx.x;
    if (j >= n)
        return;
    const int istar = *istar_p;
    double s = 0.0;
    for (int64_t k = colptr[j]; k < colptr[j + 1]; ++k)
        s = fma(u[rowidx[k]], (double)cval[k], s);
    if (istar >= 0)
        s = fma(u[istar], (double)val[(int64_t)istar * n + j], s);
    d[j] = s;
}

__global__ __launch_bounds__(WNT) void k_wide_stop1_rows(int64_t m, int nb, int G,
                                                         const double *__restrict__ rsb,
                                                         const double *__restrict__ a,
                                                         double *__restrict__ z,
                                                         double *__restrict__ rowpart)
{
    __shared__ double lds[WNT];
    int64_t i0, i1;
    part_rows(m, blockIdx.x, G, i0, i1);
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += WNT) {
        double rs = 0.0;
        for (int b = 0; b < nb; ++b)
            rs += rsb[b * m + i];
        z[i] = fmin(a[i] / rs, 1.0);
        acc += (rs - a[i]) * (rs - a[i]);
    }
    const double t = wsum(acc, lds);
    if (threadIdx.x == 0)
        rowpart[blockIdx.x] = t;
}

__global__ __launch_bounds__(WNT) void k_wide_stop2a_rows(int64_t m, int nb, int G,
                                                          const double *__restrict__ rr,
                                                          const double *__restrict__ a,
                                                          const double *__restrict__ z,
                                                          double *__restrict__ er,
                                                          double *__restrict__ zg,
                                                          double *__restrict__ rowpart)
{
    __shared__ double lds[WNT];
    int64_t i0, i1;
    part_rows(m, blockIdx.x, G, i0, i1);
    double azg = 0.0, azp = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += WNT) {
        double xy = 0.0, mg = INFINITY, mp = INFINITY;
        for (int b = 0; b < nb; ++b) {
            const double *p = rr + 3 * m * b;
            xy += p[i];
            mg = fmin(mg, p[m + i]);
            mp = fmin(mp, p[2 * m + i]);
        }
        er[i] = fmax(a[i] - z[i] * xy, 0.0);
        zg[i] = mg;
        azg += a[i] * mg;
        azp += a[i] * mp;
    }
    const double tg = wsum(azg, lds);
    const double tp = wsum(azp, lds);
    if (threadIdx.x == 0) {
        double *o = rowpart + (int64_t)blockIdx.x * STOP2_NSLOT;
        o[STOP2_AZG] = tg;
        o[STOP2_AZP] = tp;
    }
}

}  // namespace

hipError_t launch_wide_eval_rows(int64_t m, int nb, const double *Mb, const double *Sb,
                                 const double *a, const double *r, double *M, double *S,
                                 double *lse, double *f, double *rowpart, int G, hipStream_t st)
{
    hipLaunchKernelGGL(k_wide_eval_rows, dim3(G), dim3(WNT), 0, st, m, nb, G, Mb, Sb, a, r, M, S,
                       lse, f, rowpart);
    return hipGetLastError();
}

hipError_t launch_wide_trial_rows(int64_t m, int nb, const double *rr, const double *a,
                                  const double *M, const double *scal, double qg, double *Mn,
                                  double *Sn, double *f, double *rowpart, int G, hipStream_t st)
{
    hipLaunchKernelGGL(k_wide_trial_rows, dim3(G), dim3(WNT), 0, st, m, nb, G, rr, a, M, scal, qg,
                       Mn, Sn, f, rowpart);
    return hipGetLastError();
}

hipError_t launch_wide_join(int64_t m, int64_t n, int nb, int64_t bw, const int32_t *lenb,
                            const double *ksb, const double *a, const int *istar, int32_t *col,
                            void *val, int f32, int32_t *len, double *u, hipStream_t st)
{
    const unsigned g = (unsigned)(m < 16384 ? m : 16384);
    if (f32)
        hipLaunchKernelGGL(k_wide_join<float>, dim3(g), dim3(WAVE), 0, st, m, n, nb, bw, lenb, ksb,
                           a, istar, col, (float *)val, len, u);
    else
        hipLaunchKernelGGL(k_wide_join<double>, dim3(g), dim3(WAVE), 0, st, m, n, nb, bw, lenb,
                           ksb, a, istar, col, (double *)val, len, u);
    return hipGetLastError();
}

hipError_t launch_wide_d(const CsrView &c, const double *u, double *d, hipStream_t st)
{
    const dim3 grid((unsigned)((c.n + WNT - 1) / WNT));
    if (c.f32)
        hipLaunchKernelGGL(k_wide_d<float>, grid, dim3(WNT), 0, st, c.n, c.colptr, c.rowidx,
                           (const float *)c.cval, (const float *)c.val, c.istar, u, d);
    else
        hipLaunchKernelGGL(k_wide_d<double>, grid, dim3(WNT), 0, st, c.n, c.colptr, c.rowidx,
                           (const double *)c.cval, (const double *)c.val, c.istar, u, d);
    return hipGetLastError();
}

hipError_t launch_wide_stop1_rows(int64_t m, int nb, const double *rsb, const double *a, double *z,
                                  double *rowpart, int G, hipStream_t st)
{
    hipLaunchKernelGGL(k_wide_stop1_rows, dim3(G), dim3(WNT), 0, st, m, nb, G, rsb, a, z, rowpart);
    return hipGetLastError();
}

hipError_t launch_wide_stop2a_rows(int64_t m, int nb, const double *rr, const double *a,
                                   const double *z, double *er, double *zg, double *rowpart,
                                   int G, hipStream_t st)
{
    hipLaunchKernelGGL(k_wide_stop2a_rows, dim3(G), dim3(WNT), 0, st, m, nb, G, rr, a, z, er, zg,
                       rowpart);
    return hipGetLastError();
}

}  // namespace ibsn
