// cg_persistent.hip -- conjugate gradients (Algorithm 2, step 8) for
// (H_rho + shift I) x = rhs in one cooperative launch on gfx950.
//
// Late in a solve the sparsified factor keeps a few entries per row, so one CG iteration
// moves about a megabyte: it is bound by latency, and three launches per iteration cost
// more than the work they carry.  Here every workgroup stays resident for the whole solve
// (hipLaunchCooperativeKernel refuses a grid that cannot be) and the phases of an
// iteration are separated by a grid-wide barrier instead of kernel boundaries.
//
// Two barriers per iteration.  With p = r + beta p_old formed on the fly wherever it is
// read, phase A gathers the rows, u = a.(P_rho p), and the three sums that give
//     p.(H_rho + shift I) p = (sum_j d_j p_j^2 - sum_i a_i (P_rho p)_i^2) / eta
//                             + shift sum_j p_j^2
// (H_rho = (diag(d) - P_rho^T diag(a) P_rho)/eta), so alpha is known once phase A ends.
// Phase B gathers the columns, y = (H_rho + shift I) p, and applies the update at once:
// p <- p, x += alpha p, r -= alpha y, and the partial sums of r.r.  The next phase A starts
// from beta = r.r / r.r_old.
//
// The sparse structure does not change during a solve: each workgroup copies the entries of
// its rows and columns into LDS once (when they fit in 64 KB; otherwise it reads them from
// memory each iteration), so an iteration's loads are only the vector gathers.  At
// m = n = 10^4 this took an iteration from 16.8 to 15.6 us.
//
// Grid sums are per-workgroup partials added by every workgroup in index order (the same
// value everywhere, so every workgroup takes the same decisions and leaves the loop
// together).  The barrier is an arrival counter (zeroed before the launch, never reset):
// barrier k returns once the counter reaches k * grid.  Every wave waits for its own
// stores, then one wave per workgroup releases them at device scope (the L2 of each XCD
// is written back) before arriving, and acquires after the wait, so the phase's writes of
// every workgroup are seen by every other.  A release per wave instead of per workgroup
// measured 27 us per iteration against 17 us at m = n = 10^4; 1024-thread workgroups were
// slower too.  The wait is bounded: a workgroup that waits longer than BAR_SPIN polls raises
// the error flag and leaves, so a fault in the barrier ends the kernel with an error instead
// of a hang.
#include "cg_barrier.h"
#include "ibsn_internal.h"

#include <math.h>

namespace ibsn {
namespace {

constexpr int PT = 256;                  // threads per workgroup
// Sparse structure held in LDS for the whole solve: a workgroup's row slots and column slots
// (at most CACHE_SLOTS of each) with their entries, when they fit in CACHE_BYTES.
constexpr int CACHE_SLOTS = 8 * PT;
constexpr size_t CACHE_BYTES = 64 * 1024;

struct PersistArgs {
    int m, n, maxit, star_chunk;
    const int32_t *col;
    const void *val;
    const int32_t *len;
    const int *istar_p;
    const int64_t *colptr;
    const int32_t *rowidx;
    const void *cval;
    const double *d, *a, *rhs;
    double eta, shift, tol;
    double *x, *r, *p, *au;
    double *star_part, *part_a, *part_b;   // grid, 3 grid, grid
    double *scal;                          // out: CG_IT0, CG_RR0, CG_DONE0, CG_BRK
    unsigned *bar;                         // [0] arrivals, [1] error flag
};

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// Sums of four values over the workgroup (valid in every thread), fixed order.
__device__ __forceinline__ void block_sum4(double &v0, double &v1, double &v2, double &v3,
                                           double *lds)
{
    v0 = wsum(v0);
    v1 = wsum(v1);
    v2 = wsum(v2);
    v3 = wsum(v3);
    const int w = threadIdx.x / 64;
    __syncthreads();   // lds reuse across calls
    if ((threadIdx.x & 63) == 0) {
        lds[4 * w] = v0;
        lds[4 * w + 1] = v1;
        lds[4 * w + 2] = v2;
        lds[4 * w + 3] = v3;
    }
    __syncthreads();
    v0 = lds[0];
    v1 = lds[1];
    v2 = lds[2];
    v3 = lds[3];
#pragma unroll
    for (int k = 1; k < PT / 64; ++k) {
        v0 += lds[4 * k];
        v1 += lds[4 * k + 1];
        v2 += lds[4 * k + 2];
        v3 += lds[4 * k + 3];
    }
}

// In-place exclusive prefix sum of a[0..cnt) in LDS (cnt <= 8 PT), total into a[cnt];
// every thread takes 8 consecutive values.  wt: PT/64 ints of LDS.
__device__ __forceinline__ void block_exscan(int *a, int cnt, int *wt)
{
    const int t = threadIdx.x, base = 8 * t;
    int loc[8], s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        loc[k] = s;
        s += base + k < cnt ? a[base + k] : 0;
    }
    int incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if ((t & 63) >= o)
            incl += y;
    }
    if ((t & 63) == 63)
        wt[t / 64] = incl;
    __syncthreads();
    int excl = incl - s;
    for (int w = 0; w < t / 64; ++w)
        excl += wt[w];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (base + k < cnt)
            a[base + k] = excl + loc[k];
    if (t == PT - 1)
        a[cnt] = excl + s;
    __syncthreads();
}


template <int L, typename VT>
__global__ __launch_bounds__(PT) void k_cg_persist(PersistArgs A)
{
    __shared__ double lds[4 * (PT / 64)];
    __shared__ int sflag;
    const int G = (int)gridDim.x, b = (int)blockIdx.x, t = (int)threadIdx.x;
    const int m = A.m, n = A.n;
    const VT *val = static_cast<const VT *>(A.val);
    const VT *cval = static_cast<const VT *>(A.cval);
    const int istar = *A.istar_p;
    const VT *prow = istar >= 0 ? val + (int64_t)istar * n : nullptr;
    constexpr int GPB = PT / L;   // rows (columns) per workgroup per sweep
    const int l = t % L, q = t / L;
    unsigned target = 0;

    // The workgroup's rows g = b GPB + q + k G GPB (slot k GPB + q) and columns likewise
    // keep their entries in LDS for the whole solve when they fit: the iterations then
    // gather only the vectors from memory.
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ int wt[PT / 64];
    const int KR = (m + G * GPB - 1) / (G * GPB), KC = (n + G * GPB - 1) / (G * GPB);
    const int RS = KR * GPB, CS = KC * GPB;
    int *roff = reinterpret_cast<int *>(dyn), *coff = roff + RS + 1;
    const VT *rval = nullptr, *cvl = nullptr;
    const int32_t *rcol = nullptr, *crow = nullptr;
    bool cached = false;
    if (RS <= CACHE_SLOTS && CS <= CACHE_SLOTS) {
        for (int r = t; r < RS; r += PT) {
            const int g = b * GPB + (r % GPB) + (r / GPB) * G * GPB;
            roff[r] = (g < m && g != istar) ? A.len[g] : 0;
        }
        for (int r = t; r < CS; r += PT) {
            const int j = b * GPB + (r % GPB) + (r / GPB) * G * GPB;
            coff[r] = j < n ? (int)(A.colptr[j + 1] - A.colptr[j]) : 0;
        }
        __syncthreads();
        block_exscan(roff, RS, wt);
        block_exscan(coff, CS, wt);
        const int TR = roff[RS], TC = coff[CS];
        const size_t hdr = ((size_t)(RS + CS + 2) * 4 + 15) / 16 * 16;
        const size_t vbytes = ((size_t)(TR + TC) * sizeof(VT) + 15) / 16 * 16;
        cached = hdr + vbytes + (size_t)(TR + TC) * 4 <= CACHE_BYTES;
        if (cached) {
            VT *rv = reinterpret_cast<VT *>(dyn + hdr);
            VT *cv = rv + TR;
            int32_t *rc = reinterpret_cast<int32_t *>(dyn + hdr + vbytes);
            int32_t *cc = rc + TR;
            for (int k = 0; k < KR; ++k) {
                const int r = k * GPB + q, g = b * GPB + q + k * G * GPB;
                const int o = roff[r], len = roff[r + 1] - o;
                for (int e = l; e < len; e += L) {
                    rc[o + e] = A.col[(int64_t)g * n + e];
                    rv[o + e] = val[(int64_t)g * n + e];
                }
            }
            for (int k = 0; k < KC; ++k) {
                const int r = k * GPB + q, j = b * GPB + q + k * G * GPB;
                const int o = coff[r], len = coff[r + 1] - o;
                const int64_t e0 = len > 0 ? A.colptr[j] : 0;
                for (int e = l; e < len; e += L) {
                    cc[o + e] = A.rowidx[e0 + e];
                    cv[o + e] = cval[e0 + e];
                }
            }
            rval = rv;
            cvl = cv;
            rcol = rc;
            crow = cc;
        }
        __syncthreads();
    }

    // x = 0, r = rhs, p = 0 (the first iteration forms p = r + 0 p); partials of r.r
    {
        double s0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
        for (int j = b * PT + t; j < n; j += G * PT) {
            const double v = A.rhs[j];
            A.x[j] = 0.0;
            A.r[j] = v;
            A.p[j] = 0.0;
            s0 = fma(v, v, s0);
        }
        block_sum4(s0, z1, z2, z3, lds);
        if (t == 0)
            A.part_b[b] = s0;
    }
    target += (unsigned)G;
    if (!grid_barrier(A.bar, target, &sflag))
        return;

    double rr = 0.0, rr_old = 1.0;
    int it = 0;
    bool brk = false;
    for (;; ++it) {
        // ---- phase A: beta, the rows u = a.(P p), the sums of p.(H + shift) p
        {
            double q0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
            for (int k = t; k < G; k += PT)
                q0 += A.part_b[k];
            block_sum4(q0, z1, z2, z3, lds);
            rr = q0;
        }
        if (!(sqrt(rr) > A.tol) || it >= A.maxit)
            break;
        const double beta = it == 0 ? 0.0 : rr / rr_old;
        double cd = 0.0, cp = 0.0, ca = 0.0, cs = 0.0;
        for (int j = b * PT + t; j < n; j += G * PT) {
            const double pj = fma(beta, A.p[j], A.r[j]);
            const double pp = pj * pj;
            cd = fma(A.d[j], pp, cd);
            cp += pp;
        }
        if (prow) {
            const int j0 = b * A.star_chunk, j1 = min(n, j0 + A.star_chunk);
            for (int j = j0 + t; j < j1; j += PT)
                cs = fma((double)prow[j], fma(beta, A.p[j], A.r[j]), cs);
        }
        for (int k = 0; k < KR; ++k) {
            const int g = b * GPB + q + k * G * GPB;
            if (g >= m || g == istar)
                continue;   // the whole lane group skips together
            double s = 0.0;
            if (cached) {
                const int r = k * GPB + q;
                for (int e = roff[r] + l; e < roff[r + 1]; e += L) {
                    const int j = rcol[e];
                    s = fma((double)rval[e], fma(beta, A.p[j], A.r[j]), s);
                }
            } else {
                const int len = A.len[g];
                const int32_t *cr = A.col + (int64_t)g * n;
                const VT *vr = val + (int64_t)g * n;
                for (int e = l; e < len; e += L) {
                    const int j = cr[e];
                    s = fma((double)vr[e], fma(beta, A.p[j], A.r[j]), s);
                }
            }
#pragma unroll
            for (int o = L / 2; o > 0; o >>= 1)
                s += __shfl_xor(s, o, L);
            if (l == 0) {
                const double u = A.a[g] * s;
                A.au[g] = u;
                ca = fma(u, s, ca);
            }
        }
        block_sum4(cd, cp, ca, cs, lds);
        if (t == 0) {
            A.part_a[3 * b] = cd;
            A.part_a[3 * b + 1] = cp;
            A.part_a[3 * b + 2] = ca;
            A.star_part[b] = cs;
        }
        target += (unsigned)G;
        if (!grid_barrier(A.bar, target, &sflag))
            return;

        // ---- phase B: alpha, the columns y = (H + shift) p, x += alpha p, r -= alpha y
        double sd = 0.0, sp = 0.0, sa = 0.0, ss = 0.0;
        for (int k = t; k < G; k += PT) {
            sd += A.part_a[3 * k];
            sp += A.part_a[3 * k + 1];
            sa += A.part_a[3 * k + 2];
            ss += A.star_part[k];
        }
        block_sum4(sd, sp, sa, ss, lds);
        const double us = prow ? A.a[istar] * ss : 0.0;
        const double pap = (sd - sa - us * ss) / A.eta + A.shift * sp;
        if (!(pap > 0.0)) {
            brk = true;   // no step; CG ends with the iterate it has
            break;
        }
        const double alpha = rr / pap;
        double rs = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
        for (int k = 0; k < KC; ++k) {
            const int j = b * GPB + q + k * G * GPB;
            if (j >= n)
                continue;
            double s = 0.0;
            if (cached) {
                const int r = k * GPB + q;
                for (int e = coff[r] + l; e < coff[r + 1]; e += L)
                    s = fma((double)cvl[e], A.au[crow[e]], s);
            } else {
                const int64_t e0 = A.colptr[j], e1 = A.colptr[j + 1];
                for (int64_t e = e0 + l; e < e1; e += L)
                    s = fma((double)cval[e], A.au[A.rowidx[e]], s);
            }
#pragma unroll
            for (int o = L / 2; o > 0; o >>= 1)
                s += __shfl_xor(s, o, L);
            if (l == 0) {
                if (prow)
                    s = fma((double)prow[j], us, s);
                const double pj = fma(beta, A.p[j], A.r[j]);
                const double yj = (A.d[j] * pj - s) / A.eta + A.shift * pj;
                A.p[j] = pj;
                A.x[j] = fma(alpha, pj, A.x[j]);
                const double rj = fma(-alpha, yj, A.r[j]);
                A.r[j] = rj;
                rs = fma(rj, rj, rs);
            }
        }
        block_sum4(rs, z1, z2, z3, lds);
        if (t == 0)
            A.part_b[b] = rs;
        rr_old = rr;
        target += (unsigned)G;
        if (!grid_barrier(A.bar, target, &sflag))
            return;
    }
    if (b == 0 && t == 0) {
        A.scal[CG_IT0] = (double)it;
        A.scal[CG_RR0] = rr;
        A.scal[CG_DONE0] = 1.0;
        A.scal[CG_BRK] = brk ? 1.0 : 0.0;
    }
}

__global__ void k_cg_persist_reset(unsigned *bar)
{
    bar[0] = 0u;
    bar[1] = 0u;
}

template <int L, typename VT>
hipError_t launch_l(int grid, PersistArgs &A, hipStream_t st)
{
    void *args[] = {&A};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_cg_persist<L, VT>),
                                      dim3((unsigned)grid), dim3(PT), args, CACHE_BYTES, st);
}

}  // namespace

CgPersistPlan cg_persist_plan(int64_t m, int64_t n, int64_t nnz, int64_t istar, int num_cus,
                              int blocks)
{
    CgPersistPlan pl;
    const int64_t dense = istar >= 0 ? n : 0;
    const int64_t rows = istar >= 0 ? m - 1 : m;
    const double avg_row = rows > 0 ? (double)(nnz - dense) / (double)rows : 0.0;
    const double avg_col = n > 0 ? (double)(nnz - dense) / (double)n : 0.0;
    const double avg = avg_row > avg_col ? avg_row : avg_col;
    pl.lanes = avg >= 96.0 ? 64 : (avg >= 12.0 ? 16 : 4);
    if (blocks <= 0) {
        // two sweeps of rows (columns) per workgroup
        const int64_t per = 2 * (PT / pl.lanes);
        const int64_t mx = m > n ? m : n;
        int64_t g = (mx + per - 1) / per;
        blocks = (int)(g < num_cus ? g : num_cus);
    }
    pl.blocks = blocks < 1 ? 1 : (blocks > CG_PERSIST_MAX_GRID ? CG_PERSIST_MAX_GRID : blocks);
    return pl;
}

hipError_t launch_cg_persist(const CgPersistPlan &pl, const CsrView &c, const double *a,
                             double eta, double shift, const double *rhs, double tol, int maxit,
                             CgState &s, double *pp, hipStream_t st)
{
    const int G = pl.blocks;
    PersistArgs A;
    A.m = (int)c.m;
    A.n = (int)c.n;
    A.maxit = maxit;
    A.star_chunk = (int)((c.n + G - 1) / G);
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
    A.p = s.p;
    A.au = s.au;
    A.star_part = pp;
    A.part_a = pp + G;
    A.part_b = pp + 4 * G;
    A.scal = s.scal;
    A.bar = reinterpret_cast<unsigned *>(pp + 5 * G);
    hipLaunchKernelGGL(k_cg_persist_reset, dim3(1), dim3(1), 0, st, A.bar);
    if (c.f32) {
        if (pl.lanes == 64)
            return launch_l<64, float>(G, A, st);
        if (pl.lanes == 16)
            return launch_l<16, float>(G, A, st);
        return launch_l<4, float>(G, A, st);
    }
    if (pl.lanes == 64)
        return launch_l<64, double>(G, A, st);
    if (pl.lanes == 16)
        return launch_l<16, double>(G, A, st);
    return launch_l<4, double>(G, A, st);
}

}  // namespace ibsn
