// cg_pipe.hip -- conjugate gradients (Algorithm 2, step 8) for (H_rho + shift I) x = rhs with
// one grid-wide barrier per iteration, on gfx950.
//
// The product H_rho v = (d.v - P_rho^T diag(a) P_rho v) / eta takes two dependent sweeps
// (rows, then columns), so CG on it needs two grid-wide barriers per iteration, and late in
// a solve those barriers, not the bytes, are the iteration's cost.  With the dense row i*
// kept apart (it is a rank-one term), the rest of the product is one sparse matrix,
//     M = P'^T diag(a) P',   (M)_jk = sum_{i != i*} a_i P_ij P_ik,
// whose rows hold sum over the column j's entries of the length of their rows: a few times
// the factor's entries late in a solve.  Then
//     (H_rho + shift I) v = (d.v - M v - a_* P_* (P_* . v)) / eta + shift v
// is one sweep over the rows of M plus one scalar P_* . v, and the pipelined form of CG
// (P. Ghysels and W. Vanroose, "Hiding global synchronization latency in the preconditioned
// Conjugate Gradient algorithm", Parallel Computing 40(7), 2014; unpreconditioned) needs per
// iteration one product A w and the sums r.r, w.r (and here P_* . w), all of the same vector
// w: one barrier publishes w and the partial sums together.  The iterates equal those of CG
// in exact arithmetic; in floating point they agree to rounding (the recurrences differ).
//
// M is built once per CG solve: per column j, the count sum_{i in column j} len_i, a scan,
// and the entries (k, a_i P_ij P_ik) for i in column j (ascending) and k in row i
// (ascending), duplicates kept, so the layout and sums are deterministic.  Its size,
// sum_{i != i*} len_i^2, is formed with the factor (read back with its entry count), and the
// automatic choice takes this form only when M stays small.
//
// The kernel is a cooperative launch of `blocks` workgroups of 256 threads, L lanes per row
// of M, at most CG_PIPE_MAX_ROWS rows per lane group; the vectors of a workgroup's own rows
// (x, r, p, s, z, and d, P_* and w) stay in registers and its rows of M in LDS when they
// fit, since every barrier's acquire drops the caches.  w is published double-buffered by
// iteration parity (the product of one iteration reads w_i while the update writes
// w_{i+1}), and so are the partial sums.  The barrier is cg_barrier.h's.
#include "cg_barrier.h"
#include "ibsn_internal.h"

#include <math.h>

namespace ibsn {
namespace {

constexpr int PT = 256;

// sum over the rows != istar of len_i^2 (the entries of M), one workgroup, fixed order
__global__ __launch_bounds__(1024) void k_len_sq(int64_t m, const int32_t *__restrict__ len,
                                                 const int *__restrict__ istar_p,
                                                 int64_t *__restrict__ out)
{
    __shared__ int64_t part[1024];
    const int istar = *istar_p;
    int64_t s = 0;
    for (int64_t i = threadIdx.x; i < m; i += 1024)
        if (i != istar)
            s += (int64_t)len[i] * len[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[0] = part[0];
}

__global__ __launch_bounds__(256) void k_m_count(int64_t n, const int64_t *__restrict__ colptr,
                                                 const int32_t *__restrict__ rowidx,
                                                 const int32_t *__restrict__ len,
                                                 int64_t *__restrict__ cnt)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n)
        return;
    int64_t c = 0;
    for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e)
        c += len[rowidx[e]];
    cnt[j] = c;
}

// exclusive scan of cnt[0..n) into ptr[0..n] in one workgroup of 1024 threads (each a
// contiguous chunk), ptr[n] = total
__global__ __launch_bounds__(1024) void k_m_scan(int64_t n, const int64_t *__restrict__ cnt,
                                                 int64_t *__restrict__ ptr)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t j0 = t * per, j1 = j0 + per < n ? j0 + per : n;
    int64_t s = 0;
    for (int64_t j = j0; j < j1; ++j)
        s += cnt[j];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int k = 0; k < 1024; ++k) {
            const int64_t v = part[k];
            part[k] = acc;
            acc += v;
        }
        ptr[n] = acc;
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t j = j0; j < j1; ++j) {
        ptr[j] = acc;
        acc += cnt[j];
    }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_m_fill(int64_t n, const int64_t *__restrict__ colptr,
                                                const int32_t *__restrict__ rowidx,
                                                const VT *__restrict__ cval,
                                                const int32_t *__restrict__ col,
                                                const VT *__restrict__ val,
                                                const int32_t *__restrict__ len,
                                                const double *__restrict__ a,
                                                const int64_t *__restrict__ mptr,
                                                int32_t *__restrict__ mcol,
                                                double *__restrict__ mval)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n)
        return;
    int64_t pos = mptr[j];
    for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) {
        const int i = rowidx[e];
        const double wij = a[i] * (double)cval[e];
        const int L = len[i];
        const int32_t *cr = col + (int64_t)i * n;
        const VT *vr = val + (int64_t)i * n;
        for (int q = 0; q < L; ++q, ++pos) {
            mcol[pos] = cr[q];
            mval[pos] = wij * (double)vr[q];
        }
    }
}

struct PipeArgs {
    int n, maxit;
    const int64_t *mptr;
    const int32_t *mcol;
    const double *mval;
    const double *d, *rhs;
    const void *prow;   // the dense row P_* (n values), or null
    const double *a;
    const int *istar_p;
    double eta, shift, tol;
    double *x, *r, *p, *s, *z, *w;   // w: 2 n (by parity)
    double *part;                    // 2 parities x 3 x grid
    double *scal;
    unsigned *bar;
};

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void block_sum3(double &v0, double &v1, double &v2, double *lds)
{
    v0 = wsum(v0);
    v1 = wsum(v1);
    v2 = wsum(v2);
    const int w = threadIdx.x / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        lds[3 * w] = v0;
        lds[3 * w + 1] = v1;
        lds[3 * w + 2] = v2;
    }
    __syncthreads();
    v0 = lds[0];
    v1 = lds[1];
    v2 = lds[2];
#pragma unroll
    for (int k = 1; k < PT / 64; ++k) {
        v0 += lds[3 * k];
        v1 += lds[3 * k + 1];
        v2 += lds[3 * k + 2];
    }
}

// the sums of the grid's partials for parity `par` (every workgroup, index order)
__device__ __forceinline__ void grid_sums(const double *part, int G, int par, double &g0,
                                          double &g1, double &g2, double *lds)
{
    const double *pp = part + (int64_t)par * 3 * G;
    g0 = g1 = g2 = 0.0;
    for (int k = threadIdx.x; k < G; k += PT) {
        g0 += pp[3 * k];
        g1 += pp[3 * k + 1];
        g2 += pp[3 * k + 2];
    }
    block_sum3(g0, g1, g2, lds);
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

// The workgroup's rows j_k = b GPB + q + k G GPB (k < KR) keep x, r, p, s, z, d, P_*j and
// their own w in registers (lane 0 of the row's lane group uses them), and, when they fit in
// CACHE_BYTES of LDS, the entries of their rows of M: after each barrier's acquire an
// iteration then reads from memory only the published w and the partial sums.
constexpr size_t CACHE_BYTES = 64 * 1024;
constexpr int CACHE_ROWS = 8 * PT;

template <int L, int KR, typename VT>
__global__ __launch_bounds__(PT) void k_cg_pipe(PipeArgs A)
{
    __shared__ double lds[3 * (PT / 64)];
    __shared__ int sflag;
    __shared__ int wt[PT / 64];
    extern __shared__ __align__(16) unsigned char dyn[];
    const int G = (int)gridDim.x, b = (int)blockIdx.x, t = (int)threadIdx.x;
    const int n = A.n;
    constexpr int GPB = PT / L;
    const int l = t % L, q = t / L;
    const VT *prow = static_cast<const VT *>(A.prow);
    const int istar = *A.istar_p;
    const double as = istar >= 0 ? A.a[istar] : 0.0;
    unsigned target = 0;
    double *w0 = A.w, *w1 = A.w + n;

    // rows of M in LDS: row slot r = k GPB + q
    constexpr int RS = KR * GPB;
    static_assert(RS <= CACHE_ROWS, "row offsets of the cache");
    int *roff = reinterpret_cast<int *>(dyn);
    for (int r = t; r < RS; r += PT) {
        const int j = b * GPB + (r % GPB) + (r / GPB) * G * GPB;
        roff[r] = j < n ? (int)(A.mptr[j + 1] - A.mptr[j]) : 0;
    }
    __syncthreads();
    block_exscan(roff, RS, wt);
    const int TR = roff[RS];
    const size_t hdr = ((size_t)(RS + 1) * 4 + 15) / 16 * 16;
    const bool cached = hdr + (size_t)TR * 12 <= CACHE_BYTES;
    double *mv = reinterpret_cast<double *>(dyn + hdr);
    int32_t *mc = reinterpret_cast<int32_t *>(dyn + hdr + (size_t)TR * 8);
    if (cached) {
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int r = k * GPB + q, j = b * GPB + q + k * G * GPB;
            const int o = roff[r], len = roff[r + 1] - o;
            const int64_t e0 = len > 0 ? A.mptr[j] : 0;
            for (int e = l; e < len; e += L) {
                mc[o + e] = A.mcol[e0 + e];
                mv[o + e] = A.mval[e0 + e];
            }
        }
    }
    __syncthreads();
    // (A v)_j for own row k: (d_j v_j - (M v)_j - a_* P_*j zeta) / eta + shift v_j, the L
    // lanes of the group summing (M v)_j; valid in lane 0
    auto apply = [&](int k, int j, const double *v, double vj, double dj, double pj_star,
                     double zeta) -> double {
        double sm = 0.0;
        if (cached) {
            const int r = k * GPB + q;
            for (int e = roff[r] + l; e < roff[r + 1]; e += L)
                sm = fma(mv[e], v[mc[e]], sm);
        } else {
            for (int64_t e = A.mptr[j] + l; e < A.mptr[j + 1]; e += L)
                sm = fma(A.mval[e], v[A.mcol[e]], sm);
        }
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1)
            sm += __shfl_xor(sm, o, L);
        return (dj * vj - sm - as * pj_star * zeta) / A.eta + A.shift * vj;
    };

    double rx[KR], rr[KR], rp[KR], rs[KR], rz[KR], rd[KR], rps[KR], rw[KR];
    // x = 0, r = rhs; publish r (in w0) with the partial of P_* . r
    {
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int j = b * GPB + q + k * G * GPB;
            rx[k] = rr[k] = rp[k] = rs[k] = rz[k] = rd[k] = rps[k] = rw[k] = 0.0;
            if (j < n) {
                rr[k] = A.rhs[j];
                rd[k] = A.d[j];
                rps[k] = prow ? (double)prow[j] : 0.0;
                if (l == 0) {
                    w0[j] = rr[k];
                    c2 = fma(rps[k], rr[k], c2);
                }
            }
        }
        block_sum3(c0, c1, c2, lds);
        if (t == 0) {
            double *pp = A.part + 3 * (int64_t)b;   // parity 0
            pp[0] = c0;
            pp[1] = c1;
            pp[2] = c2;
        }
    }
    target += (unsigned)G;
    if (!grid_barrier(A.bar, target, &sflag))
        return;
    // w_0 = A r_0 (into w1), with the partials of r.r, w.r and P_* . w
    {
        double g0, g1, zeta;
        grid_sums(A.part, G, 0, g0, g1, zeta, lds);
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int j = b * GPB + q + k * G * GPB;
            if (j >= n)
                continue;
            rw[k] = apply(k, j, w0, rr[k], rd[k], rps[k], zeta);
            if (l == 0) {
                w1[j] = rw[k];
                c0 = fma(rr[k], rr[k], c0);
                c1 = fma(rw[k], rr[k], c1);
                c2 = fma(rps[k], rw[k], c2);
            }
        }
        block_sum3(c0, c1, c2, lds);
        if (t == 0) {
            double *pp = A.part + 3 * ((int64_t)G + b);   // parity 1
            pp[0] = c0;
            pp[1] = c1;
            pp[2] = c2;
        }
    }
    target += (unsigned)G;
    if (!grid_barrier(A.bar, target, &sflag))
        return;

    // iteration i reads w_i from wbuf[(i + 1) & 1] and the sums from parity (i + 1) & 1,
    // and writes w_{i+1} to wbuf[i & 1] and its sums to parity i & 1
    double gamma_old = 1.0, alpha_old = 1.0;
    int it = 0;
    bool brk = false;
    double gam = 0.0;
    for (;; ++it) {
        const int rd_ = (it + 1) & 1, wr = it & 1;
        double delta, zeta;
        grid_sums(A.part, G, rd_, gam, delta, zeta, lds);
        if (!(sqrt(gam) > A.tol) || it >= A.maxit)
            break;
        const double beta = it == 0 ? 0.0 : gam / gamma_old;
        const double den = it == 0 ? delta : delta - beta * gam / alpha_old;
        if (!(den > 0.0)) {
            brk = true;   // no step; CG ends with the iterate it has
            break;
        }
        const double alpha = gam / den;
        const double *wi = rd_ ? w1 : w0;
        double *wn = wr ? w1 : w0;
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int j = b * GPB + q + k * G * GPB;
            if (j >= n)
                continue;
            const double nj = apply(k, j, wi, rw[k], rd[k], rps[k], zeta);
            rz[k] = it == 0 ? nj : fma(beta, rz[k], nj);
            rs[k] = it == 0 ? rw[k] : fma(beta, rs[k], rw[k]);
            rp[k] = it == 0 ? rr[k] : fma(beta, rp[k], rr[k]);
            rx[k] = fma(alpha, rp[k], rx[k]);
            rr[k] = fma(-alpha, rs[k], rr[k]);
            rw[k] = fma(-alpha, rz[k], rw[k]);
            if (l == 0) {
                wn[j] = rw[k];
                c0 = fma(rr[k], rr[k], c0);
                c1 = fma(rw[k], rr[k], c1);
                c2 = fma(rps[k], rw[k], c2);
            }
        }
        block_sum3(c0, c1, c2, lds);
        if (t == 0) {
            double *pp = A.part + 3 * ((int64_t)wr * G + b);
            pp[0] = c0;
            pp[1] = c1;
            pp[2] = c2;
        }
        gamma_old = gam;
        alpha_old = alpha;
        target += (unsigned)G;
        if (!grid_barrier(A.bar, target, &sflag))
            return;
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int j = b * GPB + q + k * G * GPB;
        if (j < n && l == 0) {
            A.x[j] = rx[k];
            A.r[j] = rr[k];
        }
    }
    if (b == 0 && t == 0) {
        A.scal[CG_IT0] = (double)it;
        A.scal[CG_RR0] = gam;
        A.scal[CG_DONE0] = 1.0;
        A.scal[CG_BRK] = brk ? 1.0 : 0.0;
    }
}

__global__ void k_pipe_reset(unsigned *bar)
{
    bar[0] = 0u;
    bar[1] = 0u;
}

template <int L, int KR, typename VT>
hipError_t launch_l(int grid, PipeArgs &A, hipStream_t st)
{
    void *args[] = {&A};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_cg_pipe<L, KR, VT>),
                                      dim3((unsigned)grid), dim3(PT), args, CACHE_BYTES, st);
}

template <int L, typename VT>
hipError_t launch_kr(int grid, int kr, PipeArgs &A, hipStream_t st)
{
    if (kr <= 1)
        return launch_l<L, 1, VT>(grid, A, st);
    if (kr <= 2)
        return launch_l<L, 2, VT>(grid, A, st);
    if (kr <= 4)
        return launch_l<L, 4, VT>(grid, A, st);
    return launch_l<L, CG_PIPE_MAX_ROWS, VT>(grid, A, st);
}

}  // namespace

hipError_t launch_len_sq(int64_t m, const int32_t *len, const int *istar, int64_t *out,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_len_sq, dim3(1), dim3(1024), 0, st, m, len, istar, out);
    return hipGetLastError();
}

hipError_t launch_m_count(const CsrView &c, int64_t *cnt, int64_t *mptr, hipStream_t st)
{
    const dim3 g((unsigned)((c.n + 255) / 256));
    hipLaunchKernelGGL(k_m_count, g, dim3(256), 0, st, c.n, c.colptr, c.rowidx, c.len, cnt);
    hipLaunchKernelGGL(k_m_scan, dim3(1), dim3(1024), 0, st, c.n, cnt, mptr);
    return hipGetLastError();
}

hipError_t launch_m_fill(const CsrView &c, const double *a, const int64_t *mptr, int32_t *mcol,
                         double *mval, hipStream_t st)
{
    const dim3 g((unsigned)((c.n + 255) / 256));
    if (c.f32)
        hipLaunchKernelGGL(k_m_fill<float>, g, dim3(256), 0, st, c.n, c.colptr, c.rowidx,
                           (const float *)c.cval, c.col, (const float *)c.val, c.len, a, mptr,
                           mcol, mval);
    else
        hipLaunchKernelGGL(k_m_fill<double>, g, dim3(256), 0, st, c.n, c.colptr, c.rowidx,
                           (const double *)c.cval, c.col, (const double *)c.val, c.len, a, mptr,
                           mcol, mval);
    return hipGetLastError();
}

int cg_pipe_rows(int64_t n, int blocks, int lanes)
{
    const int64_t per = (int64_t)blocks * (PT / lanes);
    return (int)((n + per - 1) / per);
}

int cg_pipe_lanes(int64_t n, int64_t total)
{
    const double avg = n > 0 ? (double)total / (double)n : 0.0;
    return avg >= 48.0 ? 16 : 4;
}

hipError_t launch_cg_pipe(int blocks, int lanes, const CsrView &c, int64_t istar, const double *a,
                          const int64_t *mptr, const int32_t *mcol, const double *mval,
                          const double *rhs, double eta, double shift, double tol, int maxit,
                          CgState &s, double *w, double *pp, hipStream_t st)
{
    PipeArgs A;
    A.n = (int)c.n;
    A.maxit = maxit;
    A.mptr = mptr;
    A.mcol = mcol;
    A.mval = mval;
    A.d = c.d;
    A.rhs = rhs;
    // istar (host copy) selects the dense row's values; the kernel reads a_* on the device
    A.prow = istar >= 0 ? (c.f32 ? (const void *)((const float *)c.val + istar * c.n)
                                 : (const void *)((const double *)c.val + istar * c.n))
                        : nullptr;
    A.a = a;
    A.istar_p = c.istar;
    A.eta = eta;
    A.shift = shift;
    A.tol = tol;
    A.x = s.x;
    A.r = s.r;
    A.p = s.p;
    A.s = s.Ap;
    A.z = s.r2;
    A.w = w;
    A.part = pp;
    A.scal = s.scal;
    A.bar = reinterpret_cast<unsigned *>(pp + 6 * (int64_t)blocks);
    const int kr = cg_pipe_rows(c.n, blocks, lanes);
    if (kr > CG_PIPE_MAX_ROWS)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pipe_reset, dim3(1), dim3(1), 0, st, A.bar);
    if (c.f32)
        return lanes == 16 ? launch_kr<16, float>(blocks, kr, A, st)
                           : launch_kr<4, float>(blocks, kr, A, st);
    return lanes == 16 ? launch_kr<16, double>(blocks, kr, A, st)
                       : launch_kr<4, double>(blocks, kr, A, st);
}

}  // namespace ibsn
