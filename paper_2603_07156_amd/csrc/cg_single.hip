// cg_single.hip -- conjugate gradients (Algorithm 2, step 8) for (H_rho + shift I) x = rhs
// in one workgroup on gfx950.
//
// When the sparsified factor is small (late in a solve, or a small problem) a CG iteration
// carries a few hundred kilobytes, and its cost is the two grid-wide dependences of every
// iteration (rows before columns, columns before the next rows), not the bytes.  Here one
// workgroup of 1024 threads runs the whole solve on one CU: the dependences become
// workgroup barriers, p and u = a.(P_rho p) live in LDS (n + m doubles), and the factor is
// read from memory (L2) each iteration.  Needs no cooperative launch, so several contexts
// can run it at once on their own streams.
//
// Per iteration, with thread t owning the columns j = t + k 1024 (x, r, d and the dense
// row's entries of those columns in registers):
//   rows:    u_i = a_i sum_e val p[col] (rows != istar; row i* is the dense row), and
//            sum_i u_i (P p)_i
//   alpha:   p.(H_rho + shift I) p = (sum d p^2 - sum a (P p)^2 - u_* (P p)_*) / eta
//            + shift sum p^2, the sums over j carried from the step that formed p
//   columns: y_j = (d_j p_j - sum_i P_ij u_i) / eta + shift p_j, x += alpha p, r -= alpha y
//   beta:    r.r / r.r_old; p = r + beta p, with the sums over j of d p^2, p^2 and
//            P_*j p_j for the next alpha.
// Sums are wave butterflies then the 16 wave values in index order: every thread holds
// the same value, so all take the same branch and leave the loop together.
#include "ibsn_internal.h"

#include <math.h>

namespace ibsn {
namespace {

constexpr int ST = 1024;

struct SingleArgs {
    int m, n, maxit;
    const int32_t *col;
    const void *val;
    const int32_t *len;
    const int *istar_p;
    const int64_t *colptr;
    const int32_t *rowidx;
    const void *cval;
    const double *d, *a, *rhs;
    double eta, shift, tol;
    double *x, *r;
    double *scal;   // out: CG_IT0, CG_RR0, CG_DONE0, CG_BRK
};

__device__ __forceinline__ double wsum1(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// workgroup sums of up to four values (every thread gets them), fixed order
template <int K>
__device__ __forceinline__ void bsum(double *v, double *lds)
{
    constexpr int NW = ST / 64;
#pragma unroll
    for (int k = 0; k < K; ++k)
        v[k] = wsum1(v[k]);
    const int w = threadIdx.x / 64;
    __syncthreads();   // the previous sum's values may still be read
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            lds[k * NW + w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = lds[k * NW];
#pragma unroll
        for (int q = 1; q < NW; ++q)
            s += lds[k * NW + q];
        v[k] = s;
    }
}

template <int KC, typename VT>
__global__ __launch_bounds__(ST) void k_cg_single(SingleArgs A)
{
    extern __shared__ double sm[];   // p (n doubles), then u (m doubles)
    __shared__ double red[4 * (ST / 64)];
    const int t = (int)threadIdx.x, m = A.m, n = A.n;
    double *p = sm, *u = sm + n;
    const VT *val = static_cast<const VT *>(A.val);
    const VT *cval = static_cast<const VT *>(A.cval);
    const int istar = *A.istar_p;
    const VT *prow = istar >= 0 ? val + (int64_t)istar * n : nullptr;
    const double as = istar >= 0 ? A.a[istar] : 0.0;

    // x = 0, r = rhs, p = r; the sums of r.r, d p^2, p^2 and P_* p
    double x[KC], r[KC], d[KC], ps[KC];
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int j = t + k * ST;
        x[k] = 0.0;
        r[k] = 0.0;
        d[k] = 0.0;
        ps[k] = 0.0;
        if (j < n) {
            const double v = A.rhs[j];
            r[k] = v;
            d[k] = A.d[j];
            ps[k] = prow ? (double)prow[j] : 0.0;
            p[j] = v;
            const double vv = v * v;
            s4[0] += vv;
            s4[1] = fma(d[k], vv, s4[1]);
            s4[2] += vv;
            s4[3] = fma(ps[k], v, s4[3]);
        }
    }
    bsum<4>(s4, red);   // its barriers also publish p
    double rr = s4[0], cd = s4[1], cp = s4[2], cs = s4[3];
    int it = 0;
    bool brk = false;
    for (;;) {
        if (!(sqrt(rr) > A.tol) || it >= A.maxit)
            break;
        // rows: u = a.(P p) for the sparse rows
        double ca[1] = {0.0};
        for (int i = t; i < m; i += ST) {
            if (i == istar)
                continue;
            const int len = A.len[i];
            const int32_t *cr = A.col + (int64_t)i * n;
            const VT *vr = val + (int64_t)i * n;
            double s = 0.0;
            for (int e = 0; e < len; ++e)
                s = fma((double)vr[e], p[cr[e]], s);
            const double ui = A.a[i] * s;
            u[i] = ui;
            ca[0] = fma(ui, s, ca[0]);
        }
        bsum<1>(ca, red);   // its barriers also publish u
        const double us = as * cs;   // u of the dense row
        const double pap = (cd - ca[0] - us * cs) / A.eta + A.shift * cp;
        if (!(pap > 0.0)) {
            brk = true;   // no step; CG ends with the iterate it has
            break;
        }
        const double alpha = rr / pap;
        // columns: y = (H + shift) p, x += alpha p, r -= alpha y
        double rs[1] = {0.0};
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int j = t + k * ST;
            if (j < n) {
                const int64_t e1 = A.colptr[j + 1];
                double s = 0.0;
                for (int64_t e = A.colptr[j]; e < e1; ++e)
                    s = fma((double)cval[e], u[A.rowidx[e]], s);
                s = fma(ps[k], us, s);
                const double pj = p[j];
                const double yj = (d[k] * pj - s) / A.eta + A.shift * pj;
                x[k] = fma(alpha, pj, x[k]);
                r[k] = fma(-alpha, yj, r[k]);
                rs[0] = fma(r[k], r[k], rs[0]);
            }
        }
        bsum<1>(rs, red);
        ++it;
        const double beta = rs[0] / rr;
        rr = rs[0];
        if (!(sqrt(rr) > A.tol) || it >= A.maxit)
            break;
        // p = r + beta p and the sums over j for the next alpha
        double q4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const int j = t + k * ST;
            if (j < n) {
                const double pj = fma(beta, p[j], r[k]);
                p[j] = pj;
                const double pp = pj * pj;
                q4[0] = fma(d[k], pp, q4[0]);
                q4[1] += pp;
                q4[2] = fma(ps[k], pj, q4[2]);
            }
        }
        bsum<3>(q4, red);   // its barriers also publish p
        cd = q4[0];
        cp = q4[1];
        cs = q4[2];
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int j = t + k * ST;
        if (j < n) {
            A.x[j] = x[k];
            A.r[j] = r[k];
        }
    }
    if (t == 0) {
        A.scal[CG_IT0] = (double)it;
        A.scal[CG_RR0] = rr;
        A.scal[CG_DONE0] = 1.0;
        A.scal[CG_BRK] = brk ? 1.0 : 0.0;
    }
}

template <int KC>
hipError_t launch_kc(const SingleArgs &A, int f32, size_t lds, hipStream_t st)
{
    if (f32)
        hipLaunchKernelGGL((k_cg_single<KC, float>), dim3(1), dim3(ST), lds, st, A);
    else
        hipLaunchKernelGGL((k_cg_single<KC, double>), dim3(1), dim3(ST), lds, st, A);
    return hipGetLastError();
}

}  // namespace

size_t cg_single_lds(int64_t m, int64_t n)
{
    return (size_t)(m + n) * sizeof(double);
}

bool cg_single_fits(int64_t m, int64_t n, size_t max_lds)
{
    // p and u in dynamic LDS beside the 512 bytes of the sums; at most 10 columns a thread
    return n <= (int64_t)CG_SINGLE_MAX_COLS_PER_THREAD * ST &&
           cg_single_lds(m, n) + 4 * (ST / 64) * sizeof(double) <= max_lds;
}

hipError_t launch_cg_single(const CsrView &c, const double *a, double eta, double shift,
                            const double *rhs, double tol, int maxit, CgState &s, hipStream_t st)
{
    SingleArgs A;
    A.m = (int)c.m;
    A.n = (int)c.n;
    A.maxit = maxit;
    A.col = c.col;
    A.val = c.val;
    A.len = c.len;
    A.istar_p = c.istar;
    A.colptr = c.colptr;
    A.rowidx = c.rowidx;
    A.cval = c.cval;
    A.d = c.d;
    A.a = a;
    A.rhs = rhs;
    A.eta = eta;
    A.shift = shift;
    A.tol = tol;
    A.x = s.x;
    A.r = s.r;
    A.scal = s.scal;
    const size_t lds = cg_single_lds(c.m, c.n);
    const int kc = (int)((c.n + ST - 1) / ST);
    if (kc <= 1)
        return launch_kc<1>(A, c.f32, lds, st);
    if (kc <= 2)
        return launch_kc<2>(A, c.f32, lds, st);
    if (kc <= 4)
        return launch_kc<4>(A, c.f32, lds, st);
    if (kc <= 6)
        return launch_kc<6>(A, c.f32, lds, st);
    return launch_kc<CG_SINGLE_MAX_COLS_PER_THREAD>(A, c.f32, lds, st);
}

}  // namespace ibsn
