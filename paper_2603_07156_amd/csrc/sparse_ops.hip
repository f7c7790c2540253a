// sparse_ops.hip -- sparsified Hessian products, device-driven CG and the small
// vector kernels of the IBSN hot path on gfx950.
//
// The factor P_rho (Algorithm 1) is held twice:
//  - row slots: row i's kept entries at [i*n, i*n + len_i), columns ascending;
//  - columns (CSC): built by a deterministic counting sort over row blocks, so each
//    column lists its rows in ascending order on every run.
// H_rho v = (d.v - P_rho^T (a.(P_rho v)))/eta is then two gathers (rows, then columns)
// with no floating point atomics: results are reproducible bit for bit.
//
// CG runs entirely on the device: alpha, beta, the residual norm and a done flag live
// in device memory, so the host enqueues iterations without reading anything back.
// Grid-wide sums use a "last workgroup finishes" pattern: each workgroup writes a
// partial, the last to arrive (atomic ticket, device-scope fences) adds the partials in
// index order.
#include "ibsn_internal.h"
#include "solver_kernels.h"

#include <math.h>

namespace ibsn {
namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1)
        v += __shfl_xor(v, o, WAVE);
    return v;
}

// Sum over a workgroup of NT threads; result valid in every thread.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    constexpr int NW = NT / WAVE;
    v = wave_sum(v);
    const int w = threadIdx.x / WAVE;
    __syncthreads();   // lds reuse across calls
    if ((threadIdx.x & (WAVE - 1)) == 0)
        lds[w] = v;
    __syncthreads();
    double r = lds[0];
#pragma unroll
    for (int k = 1; k < NW; ++k)
        r += lds[k];
    return r;
}

// Last-workgroup-done: returns true in the workgroup that arrives last (all threads).
__device__ __forceinline__ bool last_block(unsigned *counter, int *flag_lds)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = atomicAdd(counter, 1u);
        *flag_lds = (t == gridDim.x - 1);
    }
    __syncthreads();
    const bool last = *flag_lds != 0;
    if (last)
        __threadfence();
    return last;
}

// ---------------------------------------------------------------------------------
// deterministic transpose of the slotted rows
// ---------------------------------------------------------------------------------
// cnt[b][j] = number of entries of column j in row block b
__global__ __launch_bounds__(256) void k_csc_count(int m, int n, int rb, const int32_t *__restrict__ col,
                                                   const int32_t *__restrict__ len,
                                                   int32_t *__restrict__ cnt)
{
    const int b = blockIdx.x;
    const int i0 = (int)((int64_t)m * b / rb), i1 = (int)((int64_t)m * (b + 1) / rb);
    int32_t *cb = cnt + (int64_t)b * n;
    for (int i = i0; i < i1; ++i) {
        const int L = len[i];
        const int32_t *cr = col + (int64_t)i * n;
        for (int e = threadIdx.x; e < L; e += blockDim.x)
            atomicAdd(&cb[cr[e]], 1);
    }
}

// per column: exclusive scan of cnt over row blocks (in place); colcnt_j = total
__global__ __launch_bounds__(256) void k_csc_blockscan(int n, int rb, int32_t *__restrict__ cnt,
                                                       int64_t *__restrict__ colcnt)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n)
        return;
    int32_t run = 0;
    for (int b = 0; b < rb; ++b) {
        const int32_t t = cnt[(int64_t)b * n + j];
        cnt[(int64_t)b * n + j] = run;
        run += t;
    }
    colcnt[j] = run;
}

// exclusive scan of n counts into ptr[0..n], single workgroup of 1024 threads;
// ptr[n] = total, also copied to *total.
__global__ __launch_bounds__(1024) void k_scan(int n, const int64_t *__restrict__ cnt,
                                               int64_t *__restrict__ ptr, int64_t *__restrict__ total)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int j0 = t * per, j1 = min(n, j0 + per);
    int64_t s = 0;
    for (int j = j0; j < j1; ++j)
        s += cnt[j];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int k = 0; k < 1024; ++k) {
            const int64_t v = part[k];
            part[k] = run;
            run += v;
        }
        ptr[n] = run;
        if (total)
            *total = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int j = j0; j < j1; ++j) {
        ptr[j] = run;
        run += cnt[j];
    }
}

// int32 counts variant (row lengths -> row_ptr)
__global__ __launch_bounds__(1024) void k_scan32(int n, const int32_t *__restrict__ cnt,
                                                 int64_t *__restrict__ ptr)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int j0 = t * per, j1 = min(n, j0 + per);
    int64_t s = 0;
    for (int j = j0; j < j1; ++j)
        s += cnt[j];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int k = 0; k < 1024; ++k) {
            const int64_t v = part[k];
            part[k] = run;
            run += v;
        }
        ptr[n] = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int j = j0; j < j1; ++j) {
        ptr[j] = run;
        run += cnt[j];
    }
}

// fill: row block b walks its rows in order; within a row every column occurs once, so
// the per-(block, column) cursor needs no atomics; rows are separated by barriers.
__global__ __launch_bounds__(256) void k_csc_fill(int m, int n, int rb, const int32_t *__restrict__ col,
                                                  const double *__restrict__ val,
                                                  const int32_t *__restrict__ len,
                                                  const int64_t *__restrict__ colptr,
                                                  int32_t *__restrict__ cur,
                                                  int32_t *__restrict__ rowidx,
                                                  double *__restrict__ cval)
{
    const int b = blockIdx.x;
    const int i0 = (int)((int64_t)m * b / rb), i1 = (int)((int64_t)m * (b + 1) / rb);
    int32_t *cb = cur + (int64_t)b * n;
    for (int i = i0; i < i1; ++i) {
        const int L = len[i];
        const int32_t *cr = col + (int64_t)i * n;
        const double *vr = val + (int64_t)i * n;
        for (int e = threadIdx.x; e < L; e += blockDim.x) {
            const int j = cr[e];
            const int32_t k = cb[j];
            cb[j] = k + 1;
            const int64_t pos = colptr[j] + k;
            rowidx[pos] = i;
            cval[pos] = vr[e];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------
// HVP gathers
// ---------------------------------------------------------------------------------
// au_i = a_i * sum_e val * v[col]; LPC lanes per row; the dense row istar is done by the
// extra last workgroup with all its threads.
template <int LPC>
__global__ __launch_bounds__(256) void k_row_gather(int m, int n, const int32_t *__restrict__ col,
                                                    const double *__restrict__ val,
                                                    const int32_t *__restrict__ len,
                                                    const int *__restrict__ istar_p,
                                                    const double *__restrict__ a,
                                                    const double *__restrict__ v,
                                                    double *__restrict__ au,
                                                    const double *__restrict__ scal, int p_mode,
                                                    const double *__restrict__ r_vec)
{
    // p_mode = 1 (inside CG): the vector gathered is p_new = r + beta * p_old, formed on the
    // fly (scal[CG_BETA]); v = p_old, r_vec = r.  Skipped when CG is done.
    if (p_mode && scal[CG_DONE] != 0.0)
        return;
    const double beta = p_mode ? scal[CG_BETA] : 0.0;
    const int istar = *istar_p;
    if (blockIdx.x == gridDim.x - 1) {
        __shared__ double lds[4];
        if (istar < 0)
            return;
        const int L = len[istar];
        const int32_t *cr = col + (int64_t)istar * n;
        const double *vr = val + (int64_t)istar * n;
        double s = 0.0;
        for (int e = threadIdx.x; e < L; e += blockDim.x) {
            const int j = cr[e];
            const double vj = p_mode ? fma(beta, v[j], r_vec[j]) : v[j];
            s = fma(vr[e], vj, s);
        }
        s = block_sum<256>(s, lds);
        if (threadIdx.x == 0)
            au[istar] = a[istar] * s;
        return;
    }
    const int g = (blockIdx.x * 256 + threadIdx.x) / LPC;
    const int l = threadIdx.x % LPC;
    if (g >= m || g == istar)
        return;
    const int L = len[g];
    const int32_t *cr = col + (int64_t)g * n;
    const double *vr = val + (int64_t)g * n;
    double s = 0.0;
    for (int e = l; e < L; e += LPC) {
        const int j = cr[e];
        const double vj = p_mode ? fma(beta, v[j], r_vec[j]) : v[j];
        s = fma(vr[e], vj, s);
    }
#pragma unroll
    for (int o = LPC / 2; o > 0; o >>= 1)
        s += __shfl_xor(s, o, LPC);
    if (l == 0)
        au[g] = a[g] * s;
}

// y_j = (d_j v_j - sum_{col j} cval * au[row]) / eta + shift * v_j.
// p_mode = 1 (CG): v_j = r_j + beta p_old_j is formed here and written back to p;
// y = Ap; per-workgroup partial of p.Ap; the last workgroup computes pAp and alpha.
template <int LPC>
__global__ __launch_bounds__(256) void k_col_gather(int n, const int64_t *__restrict__ colptr,
                                                    const int32_t *__restrict__ rowidx,
                                                    const double *__restrict__ cval,
                                                    const double *__restrict__ au,
                                                    const double *__restrict__ d,
                                                    double *__restrict__ v, double eta,
                                                    double shift, double *__restrict__ y,
                                                    double *__restrict__ scal, int p_mode,
                                                    const double *__restrict__ r_vec,
                                                    double *__restrict__ partial,
                                                    unsigned *__restrict__ counter)
{
    if (p_mode && scal[CG_DONE] != 0.0)
        return;
    __shared__ double lds[4];
    __shared__ int flag;
    const int j = (blockIdx.x * 256 + threadIdx.x) / LPC;
    const int l = threadIdx.x % LPC;
    double s = 0.0;
    if (j < n) {
        const int64_t e0 = colptr[j], e1 = colptr[j + 1];
        for (int64_t e = e0 + l; e < e1; e += LPC)
            s = fma(cval[e], au[rowidx[e]], s);
    }
#pragma unroll
    for (int o = LPC / 2; o > 0; o >>= 1)
        s += __shfl_xor(s, o, LPC);
    double pap = 0.0;
    if (j < n && l == 0) {
        double vj = v[j];
        if (p_mode) {
            vj = fma(scal[CG_BETA], vj, r_vec[j]);
            v[j] = vj;
        }
        const double yj = (d[j] * vj - s) / eta + shift * vj;
        y[j] = yj;
        pap = vj * yj;
    }
    if (!p_mode)
        return;
    pap = block_sum<256>(pap, lds);
    if (threadIdx.x == 0)
        partial[blockIdx.x] = pap;
    if (last_block(counter, &flag)) {
        double t = 0.0;
        for (int k = threadIdx.x; k < (int)gridDim.x; k += 256)
            t += partial[k];
        // fixed order: strided partial sums then the workgroup reduction
        t = block_sum<256>(t, lds);
        if (threadIdx.x == 0) {
            scal[CG_PAP] = t;
            if (!(t > 0.0)) {
                scal[CG_DONE] = 1.0;
                scal[CG_ALPHA] = 0.0;
            } else {
                scal[CG_ALPHA] = scal[CG_RR] / t;
            }
            *counter = 0u;
        }
    }
}

// x += alpha p; r -= alpha Ap; rr_new; beta = rr_new/rr; done test.
__global__ __launch_bounds__(256) void k_cg_update(int n, double *__restrict__ x,
                                                   double *__restrict__ r,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ Ap,
                                                   double *__restrict__ scal,
                                                   double *__restrict__ partial,
                                                   unsigned *__restrict__ counter)
{
    if (scal[CG_DONE] != 0.0)
        return;
    __shared__ double lds[4];
    __shared__ int flag;
    const double alpha = scal[CG_ALPHA];
    double s = 0.0;
    for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
        x[j] = fma(alpha, p[j], x[j]);
        const double rj = fma(-alpha, Ap[j], r[j]);
        r[j] = rj;
        s = fma(rj, rj, s);
    }
    s = block_sum<256>(s, lds);
    if (threadIdx.x == 0)
        partial[blockIdx.x] = s;
    if (last_block(counter, &flag)) {
        double t = 0.0;
        for (int k = threadIdx.x; k < (int)gridDim.x; k += 256)
            t += partial[k];
        t = block_sum<256>(t, lds);
        if (threadIdx.x == 0) {
            const double rr = scal[CG_RR];
            scal[CG_BETA] = t / rr;
            scal[CG_RR] = t;
            const double it = scal[CG_IT] + 1.0;
            scal[CG_IT] = it;
            if (sqrt(t) <= scal[CG_TOL] || it >= scal[CG_MAXIT])
                scal[CG_DONE] = 1.0;
            *counter = 0u;
        }
    }
}

// CG start: x = 0, r = rhs, p = rhs (the first iteration forms p = r + 0*p), rr = r.r
__global__ __launch_bounds__(1024) void k_cg_init(int n, const double *__restrict__ rhs, double tol,
                                                  int maxit, double *__restrict__ x,
                                                  double *__restrict__ r, double *__restrict__ p,
                                                  double *__restrict__ scal)
{
    __shared__ double lds[16];
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += 1024) {
        const double v = rhs[j];
        x[j] = 0.0;
        r[j] = v;
        p[j] = 0.0;
        s = fma(v, v, s);
    }
    s = block_sum<1024>(s, lds);
    if (threadIdx.x == 0) {
        scal[CG_RR] = s;
        scal[CG_PAP] = 0.0;
        scal[CG_ALPHA] = 0.0;
        scal[CG_BETA] = 0.0;
        scal[CG_TOL] = tol;
        scal[CG_IT] = 0.0;
        scal[CG_MAXIT] = (double)maxit;
        scal[CG_DONE] = (sqrt(s) <= tol || maxit <= 0) ? 1.0 : 0.0;
    }
}

// ---------------------------------------------------------------------------------
// single-workgroup reductions (fixed order) and vector kernels
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_dot(int n, const double *__restrict__ x,
                                              const double *__restrict__ y, double *__restrict__ out)
{
    __shared__ double lds[16];
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += 1024)
        s = y ? fma(x[j], y[j], s) : s + x[j];
    s = block_sum<1024>(s, lds);
    if (threadIdx.x == 0)
        *out = s;
}

// w_j = grid(s_j + gamma_j / eta), grid(v) = q * rint(v / q)
__global__ __launch_bounds__(256) void k_make_w(int n, const double *__restrict__ s,
                                                const double *__restrict__ gamma, double eta,
                                                double q, double *__restrict__ w)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) {
        const double v = s[j] + (gamma ? gamma[j] / eta : 0.0);
        w[j] = q * rint(v / q);
    }
}

// standard CSR from the row slots
__global__ __launch_bounds__(256) void k_export_csr(int m, int n, const int32_t *__restrict__ col,
                                                    const double *__restrict__ val,
                                                    const int64_t *__restrict__ row_ptr,
                                                    int32_t *__restrict__ ocol,
                                                    double *__restrict__ oval)
{
    const int i = blockIdx.x;
    if (i >= m)
        return;
    const int64_t o = row_ptr[i];
    const int L = (int)(row_ptr[i + 1] - o);
    for (int e = threadIdx.x; e < L; e += 256) {
        ocol[o + e] = col[(int64_t)i * n + e];
        oval[o + e] = val[(int64_t)i * n + e];
    }
}

}  // namespace

// ---------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------
hipError_t launch_build_csc(int64_t m, int64_t n, const int32_t *col, const double *val,
                            const int32_t *len, CscWork &w, int64_t *nnz_dev, hipStream_t st)
{
    hipError_t e = sk_zero_i32((int64_t)w.rb * n, w.blkcnt, st);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_csc_count, dim3(w.rb), dim3(256), 0, st, (int)m, (int)n, w.rb, col, len,
                       w.blkcnt);
    hipLaunchKernelGGL(k_csc_blockscan, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (int)n, w.rb, w.blkcnt, w.colcnt);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, (int)n, w.colcnt, w.colptr, nnz_dev);
    hipLaunchKernelGGL(k_csc_fill, dim3(w.rb), dim3(256), 0, st, (int)m, (int)n, w.rb, col, val,
                       len, w.colptr, w.blkcnt, w.rowidx, w.cval);
    return hipGetLastError();
}

hipError_t launch_row_gather(int64_t m, int64_t n, const int32_t *col, const double *val,
                             const int32_t *len, const int *istar, const double *a, const double *v,
                             double *au, int lpc, hipStream_t st)
{
    const int blocks = (int)((m * lpc + 255) / 256) + 1;
#define G(L)                                                                                   \
    hipLaunchKernelGGL((k_row_gather<L>), dim3(blocks), dim3(256), 0, st, (int)m, (int)n, col, \
                       val, len, istar, a, v, au, (const double *)nullptr, 0,                   \
                       (const double *)nullptr)
    if (lpc >= 64)
        G(64);
    else if (lpc >= 16)
        G(16);
    else
        G(4);
#undef G
    return hipGetLastError();
}

hipError_t launch_col_gather(int64_t n, const int64_t *colptr, const int32_t *rowidx,
                             const double *cval, const double *au, const double *d,
                             const double *v, double eta, double shift, double *y, int lpc,
                             hipStream_t st)
{
    const int blocks = (int)((n * lpc + 255) / 256);
#define G(L)                                                                                       \
    hipLaunchKernelGGL((k_col_gather<L>), dim3(blocks), dim3(256), 0, st, (int)n, colptr, rowidx, \
                       cval, au, d, const_cast<double *>(v), eta, shift, y, (double *)nullptr, 0,  \
                       (const double *)nullptr, (double *)nullptr, (unsigned *)nullptr)
    if (lpc >= 64)
        G(64);
    else if (lpc >= 16)
        G(16);
    else
        G(4);
#undef G
    return hipGetLastError();
}

hipError_t launch_cg_init(int64_t n, const double *rhs, double tol, int maxit, CgState &s,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(1024), 0, st, (int)n, rhs, tol, maxit, s.x, s.r,
                       s.p, s.scal);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(int64_t m, int64_t n, const int32_t *col, const double *val,
                               const int32_t *len, const int *istar, const int64_t *colptr,
                               const int32_t *rowidx, const double *cval, const double *d,
                               const double *a, double eta, double shift, CgState &s, int lpc_row,
                               int lpc_col, hipStream_t st)
{
    // 1) au = a . (P_rho p_new), p_new = r + beta p formed on the fly
    {
        const int blocks = (int)((m * lpc_row + 255) / 256) + 1;
#define G(L)                                                                                      \
    hipLaunchKernelGGL((k_row_gather<L>), dim3(blocks), dim3(256), 0, st, (int)m, (int)n, col, val, \
                       len, istar, a, s.p, s.au, s.scal, 1, s.r)
        if (lpc_row >= 64)
            G(64);
        else if (lpc_row >= 16)
            G(16);
        else
            G(4);
#undef G
    }
    // 2) p = p_new; Ap; pAp; alpha
    {
        const int blocks = (int)((n * lpc_col + 255) / 256);
#define G(L)                                                                                       \
    hipLaunchKernelGGL((k_col_gather<L>), dim3(blocks), dim3(256), 0, st, (int)n, colptr, rowidx, \
                       cval, s.au, d, s.p, eta, shift, s.Ap, s.scal, 1, s.r, s.partial,            \
                       s.counter)
        if (lpc_col >= 64)
            G(64);
        else if (lpc_col >= 16)
            G(16);
        else
            G(4);
#undef G
    }
    // 3) x, r, rr, beta, done
    {
        int blocks = (int)((n + 255) / 256);
        if (blocks > 256)
            blocks = 256;
        hipLaunchKernelGGL(k_cg_update, dim3(blocks), dim3(256), 0, st, (int)n, s.x, s.r, s.p,
                           s.Ap, s.scal, s.partial, s.counter + 1);
    }
    return hipGetLastError();
}

hipError_t launch_make_w(const double *s, const double *gamma, double q, double eta, int64_t n,
                         double *w, hipStream_t st)
{
    hipLaunchKernelGGL(k_make_w, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (int)n, s,
                       gamma, eta, q, w);
    return hipGetLastError();
}

hipError_t launch_sum(const double *x, int64_t n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_dot, dim3(1), dim3(1024), 0, st, (int)n, x, (const double *)nullptr, out);
    return hipGetLastError();
}

hipError_t launch_dot(const double *x, const double *y, int64_t n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_dot, dim3(1), dim3(1024), 0, st, (int)n, x, y, out);
    return hipGetLastError();
}

hipError_t launch_export_csr(int64_t m, int64_t n, const int32_t *col, const double *val,
                             const int32_t *len, int64_t *row_ptr, int32_t *ocol, double *oval,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_scan32, dim3(1), dim3(1024), 0, st, (int)m, len, row_ptr);
    hipLaunchKernelGGL(k_export_csr, dim3((unsigned)m), dim3(256), 0, st, (int)m, (int)n, col, val,
                       row_ptr, ocol, oval);
    return hipGetLastError();
}

}  // namespace ibsn
