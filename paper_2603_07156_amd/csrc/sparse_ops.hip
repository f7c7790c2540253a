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
// A grid-wide sum is a per-workgroup partial written by one kernel and added, in index
// order, by every workgroup of the next kernel that needs it (no atomics, no fences).
#include "ibsn_internal.h"
#include "solver_kernels.h"

#include <math.h>

#include <algorithm>

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

// ---------------------------------------------------------------------------------
// deterministic transpose of the slotted rows (the dense row istar is not included:
// the column gather reads it directly from its row slot, where it is stored whole in
// column order)
//
// Rows are grouped in blocks of CSC_RB = 32.  For block b and column j, bit r of
// mask[b][j] says that row 32 b + r keeps column j.  The position of entry (i, j) in
// column j is then
//     colptr[j] + off[b][j] + popcount(mask[b][j] & ((1 << r) - 1)),
// with off the exclusive scan over blocks of the mask popcounts, which lists every
// column's rows in ascending order; the fill needs no ordering between threads.
// ---------------------------------------------------------------------------------
constexpr int CSC_RB = 32;

// mask[b][j]: one workgroup per row block, masks built in LDS (n words) with atomic ORs
// (order-free), then written out.
__global__ __launch_bounds__(256) void k_csc_mask(int m, int n, const int32_t *__restrict__ col,
                                                  const int32_t *__restrict__ len,
                                                  const int *__restrict__ istar_p,
                                                  uint32_t *__restrict__ mask)
{
    extern __shared__ uint32_t mk[];
    const int b = blockIdx.x;
    const int i0 = b * CSC_RB, i1 = min(m, i0 + CSC_RB);
    for (int j = threadIdx.x; j < n; j += 256)
        mk[j] = 0u;
    __syncthreads();
    const int istar = *istar_p;
    const int wv = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    for (int i = i0 + wv; i < i1; i += 256 / WAVE) {
        if (i == istar)
            continue;
        const int L = len[i];
        const int32_t *cr = col + (int64_t)i * n;
        const uint32_t bit = 1u << (i - i0);
        for (int e = lane; e < L; e += WAVE)
            atomicOr(&mk[cr[e]], bit);
    }
    __syncthreads();
    uint32_t *mb = mask + (int64_t)b * n;
    for (int j = threadIdx.x; j < n; j += 256)
        mb[j] = mk[j];
}

// per column: off[b][j] = number of kept rows of column j in blocks before b;
// colcnt_j = total.
__global__ __launch_bounds__(256) void k_csc_blockscan(int n, int rb,
                                                       const uint32_t *__restrict__ mask,
                                                       int32_t *__restrict__ off,
                                                       int64_t *__restrict__ colcnt)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n)
        return;
    constexpr int U = 16;
    int32_t run = 0;
    int b = 0;
    for (; b + U <= rb; b += U) {
        uint32_t t[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            t[u] = mask[(int64_t)(b + u) * n + j];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            off[(int64_t)(b + u) * n + j] = run;
            run += __popc(t[u]);
        }
    }
    for (; b < rb; ++b) {
        const uint32_t t = mask[(int64_t)b * n + j];
        off[(int64_t)b * n + j] = run;
        run += __popc(t);
    }
    colcnt[j] = run;
}

// Exclusive prefix sum of one value per thread over a 1024-thread workgroup: shuffle scan
// inside each wave, then wave 0 scans the 16 wave totals.  *total receives the sum.
// Integer, so the result does not depend on the order.
__device__ __forceinline__ int64_t block_excl_scan_1024(int64_t v, int64_t *wtot, int64_t *total)
{
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const int64_t y = __shfl_up(x, o, WAVE);
        if (lane >= o)
            x += y;
    }
    if (lane == WAVE - 1)
        wtot[w] = x;
    __syncthreads();
    if (w == 0) {
        int64_t t = lane < 16 ? wtot[lane] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int64_t y = __shfl_up(t, o, WAVE);
            if (lane >= o)
                t += y;
        }
        if (lane < 16)
            wtot[lane] = t;   // inclusive totals of waves 0..lane
    }
    __syncthreads();
    *total = wtot[15];
    return (w > 0 ? wtot[w - 1] : 0) + x - v;
}

// exclusive scan of n counts into ptr[0..n], single workgroup of 1024 threads;
// ptr[n] = total.  *total = ptr[n] plus the length of the dense row istar (held in the
// row slots only), i.e. the number of stored entries of the factor.
__global__ __launch_bounds__(1024) void k_scan(int n, const int64_t *__restrict__ cnt,
                                               int64_t *__restrict__ ptr, int64_t *__restrict__ total,
                                               const int32_t *__restrict__ len,
                                               const int *__restrict__ istar_p)
{
    __shared__ int64_t wtot[16];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int j0 = t * per, j1 = min(n, j0 + per);
    int64_t s = 0;
    for (int j = j0; j < j1; ++j)
        s += cnt[j];
    int64_t all;
    int64_t run = block_excl_scan_1024(s, wtot, &all);
    if (t == 0) {
        ptr[n] = all;
        if (total) {
            const int istar = istar_p ? *istar_p : -1;
            *total = all + (istar >= 0 ? (int64_t)len[istar] : 0);
        }
    }
    for (int j = j0; j < j1; ++j) {
        ptr[j] = run;
        run += cnt[j];
    }
}

// int32 counts variant (row lengths -> row_ptr)
__global__ __launch_bounds__(1024) void k_scan32(int n, const int32_t *__restrict__ cnt,
                                                 int64_t *__restrict__ ptr)
{
    __shared__ int64_t wtot[16];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int j0 = t * per, j1 = min(n, j0 + per);
    int64_t s = 0;
    for (int j = j0; j < j1; ++j)
        s += cnt[j];
    int64_t all;
    int64_t run = block_excl_scan_1024(s, wtot, &all);
    if (t == 0)
        ptr[n] = all;
    for (int j = j0; j < j1; ++j) {
        ptr[j] = run;
        run += cnt[j];
    }
}

// Two fills write the same transpose (the position formula above); the factor's stored
// entries, known on the device once the column pointers are scanned, choose between them:
// one entry at a time while the factor is sparse, by row block from big_at entries on
// (CSC_FILL_ENTRY or CSC_FILL_BLOCK force one).  Both are launched; the other returns.
__device__ __forceinline__ bool csc_by_block(int mode, int64_t total, int64_t big_at)
{
    return mode == CSC_FILL_BLOCK || (mode == CSC_FILL_AUTO && total >= big_at);
}

// fill: LPC lanes per row, every entry independently
template <int LPC, typename VT>
__global__ __launch_bounds__(256) void k_csc_fill(int m, int n, const int32_t *__restrict__ col,
                                                  const VT *__restrict__ val,
                                                  const int32_t *__restrict__ len,
                                                  const int *__restrict__ istar_p,
                                                  const int64_t *__restrict__ colptr,
                                                  const uint32_t *__restrict__ mask,
                                                  const int32_t *__restrict__ off,
                                                  const int64_t *__restrict__ total,
                                                  int64_t big_at, int mode,
                                                  int32_t *__restrict__ rowidx,
                                                  VT *__restrict__ cval)
{
    if (csc_by_block(mode, *total, big_at))
        return;
    const int i = (blockIdx.x * 256 + threadIdx.x) / LPC;
    const int l = threadIdx.x % LPC;
    if (i >= m || i == *istar_p)
        return;
    const int L = len[i];
    const int32_t *cr = col + (int64_t)i * n;
    const VT *vr = val + (int64_t)i * n;
    const int b = i / CSC_RB;
    const uint32_t below = (1u << (i - b * CSC_RB)) - 1u;
    const uint32_t *mb = mask + (int64_t)b * n;
    const int32_t *ob = off + (int64_t)b * n;
    for (int e = l; e < L; e += LPC) {
        const int j = cr[e];
        const int64_t pos = colptr[j] + ob[j] + __popc(mb[j] & below);
        rowidx[pos] = i;
        cval[pos] = vr[e];
    }
}

// fill by row block, for factors with many entries per row: workgroup (b, y) takes the rows
// of block b and the columns [y CSC_CHUNK, (y + 1) CSC_CHUNK), in tiles of CSC_TILE.  Each
// row's entries in a tile (a run of its ascending slot, from a cursor kept per row and
// started by a binary search for the chunk's first column) are staged in LDS at (column,
// row); then thread (c, r) writes the entry of row r in column j0 + c, if the row keeps it,
// so that the block's entries of a column go out as one contiguous run where the per-entry
// fill scatters them one by one.  Wave w stages rows w CSC_RPW .. w CSC_RPW + CSC_RPW - 1,
// all of their windows of WAVE entries loaded before any is used.
constexpr int CSC_TILE = 128;
constexpr int CSC_CHUNK = 1024;
constexpr int CSC_RPW = CSC_RB / (256 / WAVE);

template <typename VT>
__global__ __launch_bounds__(256) void k_csc_fill_block(int m, int n,
                                                        const int32_t *__restrict__ col,
                                                        const VT *__restrict__ val,
                                                        const int32_t *__restrict__ len,
                                                        const int *__restrict__ istar_p,
                                                        const int64_t *__restrict__ colptr,
                                                        const uint32_t *__restrict__ mask,
                                                        const int32_t *__restrict__ off,
                                                        const int64_t *__restrict__ total,
                                                        int64_t big_at, int mode,
                                                        int32_t *__restrict__ rowidx,
                                                        VT *__restrict__ cval)
{
    if (!csc_by_block(mode, *total, big_at))
        return;
    extern __shared__ __align__(16) unsigned char csc_lds[];
    VT *tile = reinterpret_cast<VT *>(csc_lds);   // [column in tile][row in block]
    __shared__ int start[CSC_RB];
    const int b = blockIdx.x, i0 = b * CSC_RB;
    const int jb = (int)blockIdx.y * CSC_CHUNK, je = min(n, jb + CSC_CHUNK);
    const int istar = *istar_p;
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int rw0 = wv * CSC_RPW;   // the wave's first row in the block
    // each row's first entry with a column >= jb
    if (threadIdx.x < CSC_RB) {
        const int i = i0 + (int)threadIdx.x;
        int lo = 0, hi = 0;
        if (i < m && i != istar) {
            hi = len[i];
            const int32_t *cr = col + (int64_t)i * n;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (cr[mid] < jb)
                    lo = mid + 1;
                else
                    hi = mid;
            }
        }
        start[threadIdx.x] = lo;
    }
    __syncthreads();
    const uint32_t *mb = mask + (int64_t)b * n;
    const int32_t *ob = off + (int64_t)b * n;
    // per row: entries consumed so far (all with columns below the current tile) and length;
    // the same in every lane
    int cur[CSC_RPW], rl[CSC_RPW];
#pragma unroll
    for (int k = 0; k < CSC_RPW; ++k) {
        const int i = i0 + rw0 + k;
        cur[k] = start[rw0 + k];
        rl[k] = (i < m && i != istar) ? len[i] : 0;
    }
    const int r = threadIdx.x % CSC_RB;
    const uint32_t below = (1u << r) - 1u;
    for (int j0 = jb; j0 < je; j0 += CSC_TILE) {
        const int j1 = min(je, j0 + CSC_TILE);
        // stage: the entries with columns in [j0, j1) are a prefix of each row's remainder
        bool more = true;
        while (more) {
            more = false;
            int cj[CSC_RPW];
#pragma unroll
            for (int k = 0; k < CSC_RPW; ++k) {
                const int e = cur[k] + lane;
                cj[k] = e < rl[k] ? col[(int64_t)(i0 + rw0 + k) * n + e] : n;
            }
#pragma unroll
            for (int k = 0; k < CSC_RPW; ++k) {
                const bool in = cj[k] < j1;
                if (in)
                    tile[(cj[k] - j0) * CSC_RB + rw0 + k] =
                        val[(int64_t)(i0 + rw0 + k) * n + cur[k] + lane];
                const int cnt = (int)__popcll(__ballot(in));
                cur[k] += cnt;
                more |= cnt == WAVE;
            }
        }
        __syncthreads();
        // write: 256 / CSC_RB columns per pass, the rows of a column in consecutive lanes
        for (int c = threadIdx.x / CSC_RB; c < j1 - j0; c += 256 / CSC_RB) {
            const int j = j0 + c;
            const uint32_t mk = mb[j];
            if ((mk >> r) & 1u) {
                const int64_t pos = colptr[j] + ob[j] + __popc(mk & below);
                rowidx[pos] = i0 + r;
                cval[pos] = tile[c * CSC_RB + r];
            }
        }
        __syncthreads();   // the tile is staged again
    }
}

// ---------------------------------------------------------------------------------
// HVP gathers and device-driven CG
// ---------------------------------------------------------------------------------
// CG scalars are double-buffered by iteration parity: the kernels of iteration `it`
// read slot it&1 (or (it-1)&1) and only workgroup 0 of the row gather writes slot it&1,
// before any later kernel reads it.  Grid-wide sums are not finished by one workgroup:
// every consumer workgroup adds the producer's per-workgroup partials itself, in index
// order, so all of them hold the same value and no device-scope fence is needed.
//
// cg_begin (all threads of an NT-thread workgroup) returns true when CG has finished
// before iteration `it`; otherwise beta for p = r + beta p.
template <int NT>
__device__ __forceinline__ bool cg_begin(int it, double *__restrict__ scal,
                                         const double *__restrict__ rr_part, int nrr, double *lds,
                                         double *beta_out)
{
    if (it == 0) {
        *beta_out = 0.0;
        return scal[CG_DONE0] != 0.0;
    }
    const int ps = (it - 1) & 1, cs = it & 1;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (scal[CG_DONE0 + ps] != 0.0) {
        if (lead) {
            scal[CG_RR0 + cs] = scal[CG_RR0 + ps];
            scal[CG_BETA0 + cs] = 0.0;
            scal[CG_IT0 + cs] = scal[CG_IT0 + ps];
            scal[CG_DONE0 + cs] = 1.0;
        }
        return true;
    }
    double t = 0.0;
    for (int k = threadIdx.x; k < nrr; k += NT)
        t += rr_part[k];
    const double rr = block_sum<NT>(t, lds);
    const double beta = rr / scal[CG_RR0 + ps];
    const bool brk = scal[CG_BRK] != 0.0;   // p.Ap <= 0 in iteration it-1: no step taken
    const bool done = brk || !(sqrt(rr) > scal[CG_TOL]) || (double)it >= scal[CG_MAXIT];
    if (lead) {
        scal[CG_RR0 + cs] = rr;
        scal[CG_BETA0 + cs] = beta;
        scal[CG_IT0 + cs] = (double)(brk ? it - 1 : it);
        scal[CG_DONE0 + cs] = done ? 1.0 : 0.0;
    }
    *beta_out = beta;
    return done;
}

// State after `it` iterations into slot it&1 (one workgroup; the host reads it).
__global__ __launch_bounds__(256) void k_cg_check(int it, double *__restrict__ scal,
                                                  const double *__restrict__ rr_part, int nrr)
{
    __shared__ double lds[4];
    double beta;
    (void)cg_begin<256>(it, scal, rr_part, nrr, lds, &beta);
}

// au_i = a_i * sum_e val * v[col] for rows i != istar, LPC lanes per row.  The dense
// row istar (every column, in order) is split into chunks of `star_chunk` columns, one
// per extra workgroup: star_part[c] = sum over the chunk of val * v.
// CG mode (scal != null): the vector is p = r + beta p_old, formed on the fly.
template <int LPC, typename VT>
__global__ __launch_bounds__(256) void k_row_gather(int m, int n, const int32_t *__restrict__ col,
                                                    const VT *__restrict__ val,
                                                    const int32_t *__restrict__ len,
                                                    const int *__restrict__ istar_p,
                                                    const double *__restrict__ a,
                                                    const double *__restrict__ v,
                                                    double *__restrict__ au,
                                                    double *__restrict__ star_part, int row_blocks,
                                                    int star_chunk, int it,
                                                    double *__restrict__ scal,
                                                    const double *__restrict__ rr_part, int nrr,
                                                    const double *__restrict__ r_vec)
{
    __shared__ double lds[4];
    const bool cgm = scal != nullptr;
    double beta = 0.0;
    if (cgm && cg_begin<256>(it, scal, rr_part, nrr, lds, &beta))
        return;
    const int istar = *istar_p;
    if ((int)blockIdx.x >= row_blocks) {
        const int c = blockIdx.x - row_blocks;
        double s = 0.0;
        if (istar >= 0) {
            const int j0 = c * star_chunk, j1 = min(n, j0 + star_chunk);
            const VT *vr = val + (int64_t)istar * n;
            for (int j = j0 + threadIdx.x; j < j1; j += 256) {
                const double vj = cgm ? fma(beta, v[j], r_vec[j]) : v[j];
                s = fma((double)vr[j], vj, s);
            }
        }
        s = block_sum<256>(s, lds);
        if (threadIdx.x == 0)
            star_part[c] = s;
        return;
    }
    const int g = (blockIdx.x * 256 + threadIdx.x) / LPC;
    const int l = threadIdx.x % LPC;
    if (g >= m || g == istar)
        return;
    const int L = len[g];
    const int32_t *cr = col + (int64_t)g * n;
    const VT *vr = val + (int64_t)g * n;
    double s = 0.0;
    for (int e = l; e < L; e += LPC) {
        const int j = cr[e];
        const double vj = cgm ? fma(beta, v[j], r_vec[j]) : v[j];
        s = fma((double)vr[e], vj, s);
    }
#pragma unroll
    for (int o = LPC / 2; o > 0; o >>= 1)
        s += __shfl_xor(s, o, LPC);
    if (l == 0)
        au[g] = a[g] * s;
}

// y_j = (d_j v_j - sum_{i != istar} P_ij au_i - P_istar,j au_istar) / eta + shift * v_j,
// au_istar = a_istar * (sum of the dense-row chunk partials, in order).  Columns are
// taken grid-stride, LPC lanes each.
// CG mode: v_j = r_j + beta p_old_j is formed here and written back to p; y = Ap and a
// per-workgroup partial of p.Ap goes to pap_part.
template <int LPC, typename VT>
__global__ __launch_bounds__(256) void k_col_gather(int n, const int64_t *__restrict__ colptr,
                                                    const int32_t *__restrict__ rowidx,
                                                    const VT *__restrict__ cval,
                                                    const double *__restrict__ au,
                                                    const double *__restrict__ d,
                                                    const VT *__restrict__ val,
                                                    const int *__restrict__ istar_p,
                                                    const double *__restrict__ a,
                                                    const double *__restrict__ star_part,
                                                    int nstar, double *__restrict__ v, double eta,
                                                    double shift, double *__restrict__ y, int it,
                                                    const double *__restrict__ scal,
                                                    const double *__restrict__ r_vec,
                                                    double *__restrict__ pap_part)
{
    __shared__ double lds[4];
    const bool cgm = scal != nullptr;
    double beta = 0.0;
    if (cgm) {
        const int cs = it & 1;
        if (scal[CG_DONE0 + cs] != 0.0)
            return;
        beta = scal[CG_BETA0 + cs];
    }
    const int istar = *istar_p;
    double aus = 0.0;
    const VT *prow = nullptr;
    if (istar >= 0) {
        double t = 0.0;
        for (int k = threadIdx.x; k < nstar; k += 256)
            t += star_part[k];
        aus = a[istar] * block_sum<256>(t, lds);
        prow = val + (int64_t)istar * n;
    }
    constexpr int CPB = 256 / LPC;
    const int l = threadIdx.x % LPC;
    double pap = 0.0;
    for (int j = blockIdx.x * CPB + threadIdx.x / LPC; j < n; j += gridDim.x * CPB) {
        const int64_t e0 = colptr[j], e1 = colptr[j + 1];
        double s = 0.0;
        for (int64_t e = e0 + l; e < e1; e += LPC)
            s = fma((double)cval[e], au[rowidx[e]], s);
#pragma unroll
        for (int o = LPC / 2; o > 0; o >>= 1)
            s += __shfl_xor(s, o, LPC);
        if (l == 0) {
            double vj = v[j];
            if (cgm) {
                vj = fma(beta, vj, r_vec[j]);
                v[j] = vj;
            }
            if (prow)
                s = fma((double)prow[j], aus, s);
            const double yj = (d[j] * vj - s) / eta + shift * vj;
            y[j] = yj;
            pap = fma(vj, yj, pap);
        }
    }
    if (!cgm)
        return;
    pap = block_sum<256>(pap, lds);
    if (threadIdx.x == 0)
        pap_part[blockIdx.x] = pap;
}

constexpr int GUNR = 8;   // loads in flight per lane in the LDS-staged gathers

template <typename VT> struct Pair2;
template <> struct Pair2<double> { using T = double2; };
template <> struct Pair2<float> { using T = float2; };

// sum_{e < L} val[e] * vec[idx[e]] over the LPC lanes of a group (lane l), entries taken in
// aligned pairs: one 8-byte index load and one 2-value load per pair, GUNR pairs in
// flight per lane.  `odd` = the global offset of entry 0 is odd: entry 0 is then taken
// alone (by lane 0) and the pairs start at entry 1; an unpaired last entry is taken alone
// by lane 0 too.  Returns the lane's partial sum (fixed order for fixed inputs).
template <int LPC, typename VT>
__device__ __forceinline__ double pair_dot(const int32_t *__restrict__ idx,
                                           const VT *__restrict__ val, int64_t L, bool odd,
                                           int l, const double *__restrict__ vec)
{
    using V2 = typename Pair2<VT>::T;
    double s = 0.0;
    const int64_t h = (odd && L > 0) ? 1 : 0;
    const int64_t npair = (L - h) >> 1;
    if (l == 0) {
        if (h)
            s = fma((double)val[0], vec[idx[0]], s);
        if (((L - h) & 1) != 0)
            s = fma((double)val[L - 1], vec[idx[L - 1]], s);
    }
    const int2 *ip = reinterpret_cast<const int2 *>(idx + h);
    const V2 *vp = reinterpret_cast<const V2 *>(val + h);
    for (int64_t base = l; base < npair; base += GUNR * LPC) {
        int2 jj[GUNR];
        V2 vv[GUNR];
#pragma unroll
        for (int k = 0; k < GUNR; ++k) {
            const int64_t p = base + k * LPC;
            if (p < npair) {
                jj[k] = ip[p];
                vv[k] = vp[p];
            } else {
                jj[k] = make_int2(0, 0);
                vv[k].x = 0;
                vv[k].y = 0;
            }
        }
#pragma unroll
        for (int k = 0; k < GUNR; ++k) {
            s = fma((double)vv[k].x, vec[jj[k].x], s);
            s = fma((double)vv[k].y, vec[jj[k].y], s);
        }
    }
    return s;
}

// dst[j] = beta * v[j] + r[j] (r null: dst[j] = v[j]) for j < len, 1024 threads, with
// sixteen independent loads in flight per thread (a plain strided loop waits on each
// load): one round of loads for len <= 16384
__device__ __forceinline__ void stage_vec(double *dst, const double *__restrict__ v,
                                          const double *__restrict__ r, double beta, int len)
{
    constexpr int U = 16;
    for (int j0 = threadIdx.x; j0 < len; j0 += U * 1024) {
        double a[U], b[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int j = j0 + k * 1024;
            a[k] = j < len ? v[j] : 0.0;
            b[k] = (r && j < len) ? r[j] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int j = j0 + k * 1024;
            if (j < len)
                dst[j] = r ? fma(beta, a[k], b[k]) : a[k];
        }
    }
}

// Star-row chunks and rows of the LDS-staged row gather, with the gathered vector already in
// vs (n doubles, visible to the whole workgroup).
template <int LPC, typename VT>
__device__ __forceinline__ void row_gather_tail(int m, int n, const int32_t *__restrict__ col,
                                                const VT *__restrict__ val,
                                                const int32_t *__restrict__ len, int istar,
                                                const double *__restrict__ a, const double *vs,
                                                double *__restrict__ au,
                                                double *__restrict__ star_part, int nstar,
                                                int star_chunk, double *lds)
{
    for (int c = blockIdx.x; c < nstar; c += gridDim.x) {
        double t = 0.0;
        if (istar >= 0) {
            const int j0 = c * star_chunk, j1 = min(n, j0 + star_chunk);
            const VT *vr = val + (int64_t)istar * n;
            for (int j = j0 + threadIdx.x; j < j1; j += 1024)
                t = fma((double)vr[j], vs[j], t);
        }
        t = block_sum<1024>(t, lds);
        if (threadIdx.x == 0)
            star_part[c] = t;
    }
    // rows interleaved over the workgroups (row g in workgroup g mod grid), so that every
    // workgroup gets an equal share even when m < grid * groups per workgroup
    constexpr int GPB = 1024 / LPC;
    const int l = threadIdx.x % LPC;
    for (int g = blockIdx.x + gridDim.x * (threadIdx.x / LPC); g < m; g += gridDim.x * GPB) {
        if (g == istar)
            continue;
        const int L = len[g];
        const int64_t off = (int64_t)g * n;
        double s = pair_dot<LPC, VT>(col + off, val + off, L, (off & 1) != 0, l, vs);
#pragma unroll
        for (int o = LPC / 2; o > 0; o >>= 1)
            s += __shfl_xor(s, o, LPC);
        if (l == 0)
            au[g] = a[g] * s;
    }
}

// The same two gathers with the gathered vector staged in LDS by every workgroup
// (n, respectively m, doubles), on a persistent grid of 1024-thread workgroups: the
// sparse entries are then read as coalesced streams of (index, value) pairs (pair_dot)
// and the vector from LDS.  Each sum has its own fixed order, so results are
// run-to-run reproducible (the order differs from the kernels above).
template <int LPC, typename VT>
__global__ __launch_bounds__(1024) void k_row_gather_lds(int m, int n,
                                                         const int32_t *__restrict__ col,
                                                         const VT *__restrict__ val,
                                                         const int32_t *__restrict__ len,
                                                         const int *__restrict__ istar_p,
                                                         const double *__restrict__ a,
                                                         const double *__restrict__ v,
                                                         double *__restrict__ au,
                                                         double *__restrict__ star_part,
                                                         int nstar, int star_chunk, int it,
                                                         double *__restrict__ scal,
                                                         const double *__restrict__ rr_part,
                                                         int nrr,
                                                         const double *__restrict__ r_vec)
{
    extern __shared__ double vs[];   // the gathered vector, n doubles
    __shared__ double lds[16];
    const bool cgm = scal != nullptr;
    double beta = 0.0;
    if (cgm && cg_begin<1024>(it, scal, rr_part, nrr, lds, &beta))
        return;
    stage_vec(vs, v, cgm ? r_vec : nullptr, beta, n);
    __syncthreads();
    row_gather_tail<LPC, VT>(m, n, col, val, len, *istar_p, a, vs, au, star_part, nstar,
                             star_chunk, lds);
}

// Two-kernel CG iteration for small n, where each kernel's work is a few microseconds
// and a third launch per iteration is a large share of the time.  Iteration `it` >= 1 of
// the row gather first finishes iteration it-1 (the vector update of the three-kernel form):
//   alpha = rr_{it-1} / p.Ap (p.Ap from the column gather's partials, added in order),
//   r_it = r_{it-1} - alpha Ap over all n in every workgroup, so that each forms the same
//   ||r_it||^2 (same order, same operations); x += alpha p and r_it are written only for
//   the workgroup's own slice of columns.  r is double-buffered by iteration parity (r_it in
//   rbuf[it & 1]), so no workgroup reads an entry another one writes.  p.Ap <= 0 (or not a
//   number): no step, and CG ends with the previous iterate, as in the three-kernel form.
// Then beta, the done test, and workgroup 0 writes slot it & 1 of the scalars.
// vs (LDS, n doubles) receives r_it.  When write_if_done_only (the single-workgroup state
// kernel), nothing is written unless CG has finished; it then writes x and r for all n.
template <int NT>
__device__ __forceinline__ bool cg_fused_update(int it, int n, double *__restrict__ scal,
                                                const double *__restrict__ pap_part, int npap,
                                                double *__restrict__ x,
                                                const double *__restrict__ rprev,
                                                double *__restrict__ rcur,
                                                const double *__restrict__ p,
                                                const double *__restrict__ Ap, double *vs,
                                                int lo, int hi, bool write_if_done_only,
                                                double *lds, double *beta_out)
{
    const int ps = (it - 1) & 1, cs = it & 1;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (scal[CG_DONE0 + ps] != 0.0) {
        if (lead) {
            scal[CG_RR0 + cs] = scal[CG_RR0 + ps];
            scal[CG_BETA0 + cs] = 0.0;
            scal[CG_IT0 + cs] = scal[CG_IT0 + ps];
            scal[CG_DONE0 + cs] = 1.0;
        }
        return true;
    }
    // The state kernel already finished iteration `it` (CG ended exactly where the host
    // polled) and wrote x, r and slot cs; a row gather queued after that poll must not
    // apply x += alpha p a second time.  The marker is written only by the state kernel,
    // never by a workgroup of the kernel that reads it.
    if (!write_if_done_only && scal[CG_FIN] == (double)it)
        return true;
    double t = 0.0;
    for (int k = threadIdx.x; k < npap; k += NT)
        t += pap_part[k];
    const double pap = block_sum<NT>(t, lds);
    const bool ok = pap > 0.0;
    const double rr_old = scal[CG_RR0 + ps];
    const double alpha = ok ? rr_old / pap : 0.0;
    double acc = 0.0;
    for (int j = threadIdx.x; j < n; j += NT) {
        const double rn = ok ? fma(-alpha, Ap[j], rprev[j]) : rprev[j];
        if (vs)
            vs[j] = rn;
        acc = fma(rn, rn, acc);
    }
    const double rr = block_sum<NT>(acc, lds);   // its barriers also publish vs
    const bool done = !ok || !(sqrt(rr) > scal[CG_TOL]) || (double)it >= scal[CG_MAXIT];
    if (!write_if_done_only || done) {
        for (int j = lo + (int)threadIdx.x; j < hi; j += NT) {
            if (ok)
                x[j] = fma(alpha, p[j], x[j]);
            rcur[j] = vs ? vs[j] : (ok ? fma(-alpha, Ap[j], rprev[j]) : rprev[j]);
        }
    }
    const double beta = rr / rr_old;
    if (lead) {
        scal[CG_RR0 + cs] = rr;
        scal[CG_BETA0 + cs] = beta;
        scal[CG_IT0 + cs] = (double)(ok ? it : it - 1);
        scal[CG_DONE0 + cs] = done ? 1.0 : 0.0;
        if (write_if_done_only && done)
            scal[CG_FIN] = (double)it;
    }
    *beta_out = beta;
    return done;
}

template <int LPC, typename VT>
__global__ __launch_bounds__(1024) void k_row_gather_cg(int m, int n,
                                                        const int32_t *__restrict__ col,
                                                        const VT *__restrict__ val,
                                                        const int32_t *__restrict__ len,
                                                        const int *__restrict__ istar_p,
                                                        const double *__restrict__ a,
                                                        double *__restrict__ au,
                                                        double *__restrict__ star_part,
                                                        int nstar, int star_chunk, int it,
                                                        double *__restrict__ scal,
                                                        const double *__restrict__ pap_part,
                                                        int npap, double *__restrict__ x,
                                                        double *__restrict__ r0,
                                                        double *__restrict__ r1,
                                                        const double *__restrict__ p,
                                                        const double *__restrict__ Ap)
{
    extern __shared__ double vs[];   // r_it, then p_it = r_it + beta p_{it-1}
    __shared__ double lds[16];
    double beta = 0.0;
    if (it == 0) {
        if (scal[CG_DONE0] != 0.0)
            return;
        for (int j = threadIdx.x; j < n; j += 1024)
            vs[j] = r0[j];   // p_0 = r_0
    } else {
        const int chunk = (n + (int)gridDim.x - 1) / (int)gridDim.x;
        const int lo = min(n, (int)blockIdx.x * chunk), hi = min(n, lo + chunk);
        double *rprev = (it & 1) ? r0 : r1, *rcur = (it & 1) ? r1 : r0;
        if (cg_fused_update<1024>(it, n, scal, pap_part, npap, x, rprev, rcur, p, Ap, vs, lo,
                                  hi, false, lds, &beta))
            return;
        __syncthreads();   // the slice writes above read r_it from vs: finish them first
        for (int j = threadIdx.x; j < n; j += 1024)
            vs[j] = fma(beta, p[j], vs[j]);
    }
    __syncthreads();
    row_gather_tail<LPC, VT>(m, n, col, val, len, *istar_p, a, vs, au, star_part, nstar,
                             star_chunk, lds);
}

// State after `it` iterations of the two-kernel CG into slot it & 1 (one workgroup; the host
// reads it).  Writes x and r only if CG has then finished (otherwise the next row gather
// performs the same update).
__global__ __launch_bounds__(1024) void k_cg_state(int it, int n, double *__restrict__ scal,
                                                   const double *__restrict__ pap_part, int npap,
                                                   double *__restrict__ x,
                                                   double *__restrict__ r0,
                                                   double *__restrict__ r1,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ Ap)
{
    __shared__ double lds[16];
    if (it == 0)
        return;   // k_cg_init wrote slot 0
    double beta;
    double *rprev = (it & 1) ? r0 : r1, *rcur = (it & 1) ? r1 : r0;
    (void)cg_fused_update<1024>(it, n, scal, pap_part, npap, x, rprev, rcur, p, Ap, nullptr, 0,
                                n, true, lds, &beta);
}

template <int LPC, typename VT>
__global__ __launch_bounds__(1024) void k_col_gather_lds(int m, int n,
                                                         const int64_t *__restrict__ colptr,
                                                         const int32_t *__restrict__ rowidx,
                                                         const VT *__restrict__ cval,
                                                         const double *__restrict__ au,
                                                         const double *__restrict__ d,
                                                         const VT *__restrict__ val,
                                                         const int *__restrict__ istar_p,
                                                         const double *__restrict__ a,
                                                         const double *__restrict__ star_part,
                                                         int nstar, double *__restrict__ v,
                                                         double eta, double shift,
                                                         double *__restrict__ y, int it,
                                                         const double *__restrict__ scal,
                                                         const double *__restrict__ r_vec,
                                                         double *__restrict__ pap_part)
{
    extern __shared__ double us[];   // a_i (P p)_i, m doubles (entry istar unused)
    __shared__ double lds[16];
    const bool cgm = scal != nullptr;
    double beta = 0.0;
    if (cgm) {
        const int cs = it & 1;
        if (scal[CG_DONE0 + cs] != 0.0)
            return;
        beta = scal[CG_BETA0 + cs];
    }
    stage_vec(us, au, nullptr, 0.0, m);
    const int istar = *istar_p;
    double aus = 0.0;
    const VT *prow = nullptr;
    double t = 0.0;
    for (int k = threadIdx.x; k < nstar; k += 1024)
        t += star_part[k];
    t = block_sum<1024>(t, lds);   // its barriers also publish us[]
    if (istar >= 0) {
        aus = a[istar] * t;
        prow = val + (int64_t)istar * n;
    }
    constexpr int CPB = 1024 / LPC;
    const int l = threadIdx.x % LPC;
    double pap = 0.0;
    for (int j = blockIdx.x + gridDim.x * (threadIdx.x / LPC); j < n; j += gridDim.x * CPB) {
        const int64_t e0 = colptr[j], e1 = colptr[j + 1];
        double s = pair_dot<LPC, VT>(rowidx + e0, cval + e0, e1 - e0, (e0 & 1) != 0, l, us);
#pragma unroll
        for (int o = LPC / 2; o > 0; o >>= 1)
            s += __shfl_xor(s, o, LPC);
        if (l == 0) {
            double vj = v[j];
            if (cgm) {
                vj = fma(beta, vj, r_vec[j]);
                v[j] = vj;
            }
            if (prow)
                s = fma((double)prow[j], aus, s);
            const double yj = (d[j] * vj - s) / eta + shift * vj;
            y[j] = yj;
            pap = fma(vj, yj, pap);
        }
    }
    if (!cgm)
        return;
    pap = block_sum<1024>(pap, lds);
    if (threadIdx.x == 0)
        pap_part[blockIdx.x] = pap;
}

// alpha = rr / p.Ap (p.Ap from the column-gather partials, in order); x += alpha p;
// r -= alpha Ap; per-workgroup partial of r.r.  p.Ap <= 0 (or not a number): no step,
// flag it for the next iteration's start.
__global__ __launch_bounds__(256) void k_cg_update(int n, int it, double *__restrict__ x,
                                                   double *__restrict__ r,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ Ap,
                                                   double *__restrict__ scal,
                                                   const double *__restrict__ pap_part, int npap,
                                                   double *__restrict__ rr_part)
{
    __shared__ double lds[4];
    const int cs = it & 1;
    if (scal[CG_DONE0 + cs] != 0.0)
        return;
    double t = 0.0;
    for (int k = threadIdx.x; k < npap; k += 256)
        t += pap_part[k];
    t = block_sum<256>(t, lds);
    const bool ok = t > 0.0;
    if (!ok && blockIdx.x == 0 && threadIdx.x == 0)
        scal[CG_BRK] = 1.0;
    const double alpha = ok ? scal[CG_RR0 + cs] / t : 0.0;
    double s = 0.0;
    for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
        double rj = r[j];
        if (ok) {
            x[j] = fma(alpha, p[j], x[j]);
            rj = fma(-alpha, Ap[j], rj);
            r[j] = rj;
        }
        s = fma(rj, rj, s);
    }
    s = block_sum<256>(s, lds);
    if (threadIdx.x == 0)
        rr_part[blockIdx.x] = s;
}

// CG start: x = 0, r = rhs, p = 0 (the first iteration forms p = r + 0*p), rr = r.r
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
        scal[CG_TOL] = tol;
        scal[CG_MAXIT] = (double)maxit;
        scal[CG_BRK] = 0.0;
        scal[CG_RR0] = s;
        scal[CG_BETA0] = 0.0;
        scal[CG_IT0] = 0.0;
        scal[CG_DONE0] = (!(sqrt(s) > tol) || maxit <= 0) ? 1.0 : 0.0;
        // slot 1 may hold the end of a previous solve
        scal[CG_RR1] = s;
        scal[CG_BETA1] = 0.0;
        scal[CG_IT1] = 0.0;
        scal[CG_DONE1] = 0.0;
        scal[CG_FIN] = -1.0;
        scal[CG_RR1] = 0.0;
        scal[CG_BETA1] = 0.0;
        scal[CG_IT1] = 0.0;
        scal[CG_DONE1] = 0.0;
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
// w = s + gamma/eta as a two-level potential: wh = grid(s + d) with d = gamma/eta rounded,
// wl = the rest, exactly up to one rounding at the size of wl: (s + d) - wh is exact, the
// error of s + d comes from a two-sum and that of d from an fma residual.  split = 0: wh =
// grid(s + gamma/eta), wl = 0 (potentials on the grid).
__global__ __launch_bounds__(256) void k_make_w(int n, const double *__restrict__ s,
                                                const double *__restrict__ gamma, double eta,
                                                double q, int split, double *__restrict__ w,
                                                double *__restrict__ wlo)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) {
        const double sj = s[j], gj = gamma ? gamma[j] : 0.0;
        const double d = gj / eta;
        const double t = sj + d;
        const double wh = q * rint(t / q);
        w[j] = wh;
        if (split) {
            const double rd = fma(-d, eta, gj);   // gamma - d eta, exactly
            const double bb = t - sj;
            const double e = (sj - (t - bb)) + (d - bb);
            wlo[j] = ((t - wh) + e) + rd / eta;
        } else {
            wlo[j] = 0.0;
        }
    }
}

// standard CSR from the row slots (values widened to FP64); writes stay below cap (the
// caller's buffer length)
template <typename VT>
__global__ __launch_bounds__(256) void k_export_csr(int m, int n, const int32_t *__restrict__ col,
                                                    const VT *__restrict__ val,
                                                    const int64_t *__restrict__ row_ptr,
                                                    int32_t *__restrict__ ocol,
                                                    double *__restrict__ oval, int64_t cap)
{
    const int i = blockIdx.x;
    if (i >= m)
        return;
    const int64_t o = row_ptr[i];
    const int L = (int)min(row_ptr[i + 1] - o, cap - o);
    for (int e = threadIdx.x; e < L; e += 256) {
        ocol[o + e] = col[(int64_t)i * n + e];
        oval[o + e] = (double)val[(int64_t)i * n + e];
    }
}

}  // namespace

// ---------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------
GatherPlan gather_plan(int64_t m, int64_t n, int64_t nnz, int64_t istar, int num_cus,
                       size_t max_lds)
{
    GatherPlan g;
    // the LDS-staged gathers hold an n-vector (rows) or an m-vector (columns) per workgroup;
    // past the size of the two-kernel form, staging pays only when each workgroup then reads
    // many entries from LDS: with fewer than about a quarter of the vector's length per
    // workgroup (a sparse late factor) the staging is most of the traffic (at 10^4 and 3.4e4
    // entries the staged gathers moved 9x the algorithmic bytes from HBM), and the gathers
    // read the vectors directly
    const int64_t dense_e = istar >= 0 ? n : 0;
    const bool enough = n <= CG_FUSED_MAX_N ||
                        (double)(nnz - dense_e) >= 0.25 * (double)num_cus * (double)std::max(m, n);
    g.lds = enough && (size_t)n * 8 + 256 <= max_lds && (size_t)m * 8 + 256 <= max_lds;
    const int64_t dense = istar >= 0 ? n : 0;
    const int64_t rows = istar >= 0 ? m - 1 : m;
    const double avg_row = rows > 0 ? (double)(nnz - dense) / (double)rows : 0.0;
    const double avg_col = n > 0 ? (double)(nnz - dense) / (double)n : 0.0;
    auto lanes = [](double avg) { return avg >= 96.0 ? 64 : (avg >= 12.0 ? 16 : 4); };
    g.lpc_row = lanes(avg_row);
    g.lpc_col = lanes(avg_col);
    if (g.lds) {
        // with the vector in LDS and GUNR loads in flight per lane, several rows per wave
        // beat one long row per wave
        g.lpc_row = avg_row >= 12.0 ? 16 : 4;
        g.lpc_col = avg_col >= 12.0 ? 16 : 4;
    }
    g.row_blocks = (int)((m * g.lpc_row + 255) / 256);
    g.star_chunk = 1024;
    g.nstar = (int)((n + g.star_chunk - 1) / g.star_chunk);
    if (g.nstar > CG_MAX_STAR) {
        g.nstar = CG_MAX_STAR;
        g.star_chunk = (int)((n + CG_MAX_STAR - 1) / CG_MAX_STAR);
    }
    const int64_t need = (n * g.lpc_col + 255) / 256;
    g.col_blocks = (int)std::min<int64_t>(need, std::min<int64_t>(CG_MAX_COLGROUPS, 4 * num_cus));
    if (g.col_blocks < 1)
        g.col_blocks = 1;
    if (g.lds) {
        g.row_blocks = num_cus;   // persistent: one 1024-thread workgroup per CU
        g.col_blocks = (int)std::min<int64_t>(num_cus, CG_MAX_COLGROUPS);
    }
    g.upd_blocks = (int)std::min<int64_t>((n + 255) / 256, CG_MAX_UPDGROUPS);
    // two kernels per CG iteration while the vector update repeated in every workgroup
    // (4 n-vectors read from L2) costs less than a third launch
    g.fused = g.lds && n <= CG_FUSED_MAX_N;
    if (g.upd_blocks < 1)
        g.upd_blocks = 1;
    return g;
}

int csc_row_blocks(int64_t m) { return (int)((m + CSC_RB - 1) / CSC_RB); }

hipError_t launch_build_csc(int64_t m, int64_t n, const int32_t *col, const void *val, int f32,
                            const int32_t *len, const int *istar, CscWork &w, int64_t *nnz_dev,
                            hipStream_t st)
{
    const int rb = csc_row_blocks(m);
    hipLaunchKernelGGL(k_csc_mask, dim3(rb), dim3(256), (size_t)n * 4, st, (int)m, (int)n, col, len,
                       istar, w.mask);
    hipLaunchKernelGGL(k_csc_blockscan, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       (int)n, rb, w.mask, w.off, w.colcnt);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, (int)n, w.colcnt, w.colptr, nnz_dev, len,
                       istar);
    const int lpc = w.lpc;
    const unsigned blocks = (unsigned)((m * lpc + 255) / 256);
    const int64_t big_at = std::max<int64_t>(1, (int64_t)(CSC_BLOCK_MIN_DENSITY * (double)m *
                                                          (double)n));
#define FILL(L_, VT_)                                                                          \
    hipLaunchKernelGGL((k_csc_fill<L_, VT_>), dim3(blocks), dim3(256), 0, st, (int)m, (int)n, col, \
                       (const VT_ *)val, len, istar, w.colptr, w.mask, w.off, nnz_dev, big_at, \
                       w.fill, w.rowidx, (VT_ *)w.cval)
#define FILLB(VT_)                                                                             \
    hipLaunchKernelGGL((k_csc_fill_block<VT_>),                                                \
                       dim3((unsigned)rb, (unsigned)((n + CSC_CHUNK - 1) / CSC_CHUNK)), dim3(256), \
                       (size_t)CSC_TILE * CSC_RB * sizeof(VT_), st, (int)m, (int)n, col,          \
                       (const VT_ *)val, len, istar, w.colptr, w.mask, w.off, nnz_dev, big_at, \
                       w.fill, w.rowidx, (VT_ *)w.cval)
    if (f32) {
        if (w.fill != CSC_FILL_BLOCK) {
            if (lpc >= 64)
                FILL(64, float);
            else
                FILL(16, float);
        }
        if (w.fill != CSC_FILL_ENTRY)
            FILLB(float);
    } else {
        if (w.fill != CSC_FILL_BLOCK) {
            if (lpc >= 64)
                FILL(64, double);
            else
                FILL(16, double);
        }
        if (w.fill != CSC_FILL_ENTRY)
            FILLB(double);
    }
#undef FILLB
#undef FILL
    return hipGetLastError();
}

namespace {
template <int L, typename VT>
void row_gather_lt(const GatherPlan &g, const CsrView &c, const double *a, const double *v,
                   double *au, double *star_part, int it, double *scal, const double *rr_part,
                   int nrr, const double *r_vec, hipStream_t st)
{
    const VT *val = (const VT *)c.val;
    if (g.lds)
        hipLaunchKernelGGL((k_row_gather_lds<L, VT>), dim3(g.row_blocks), dim3(1024),
                           (size_t)c.n * sizeof(double), st, (int)c.m, (int)c.n, c.col, val,
                           c.len, c.istar, a, v, au, star_part, g.nstar, g.star_chunk, it, scal,
                           rr_part, nrr, r_vec);
    else
        hipLaunchKernelGGL((k_row_gather<L, VT>), dim3(g.row_blocks + g.nstar), dim3(256), 0, st,
                           (int)c.m, (int)c.n, c.col, val, c.len, c.istar, a, v, au, star_part,
                           g.row_blocks, g.star_chunk, it, scal, rr_part, nrr, r_vec);
}

template <int L>
void row_gather_l(const GatherPlan &g, const CsrView &c, const double *a, const double *v,
                  double *au, double *star_part, int it, double *scal, const double *rr_part,
                  int nrr, const double *r_vec, hipStream_t st)
{
    if (c.f32)
        row_gather_lt<L, float>(g, c, a, v, au, star_part, it, scal, rr_part, nrr, r_vec, st);
    else
        row_gather_lt<L, double>(g, c, a, v, au, star_part, it, scal, rr_part, nrr, r_vec, st);
}

void row_gather(const GatherPlan &g, const CsrView &c, const double *a, const double *v,
                double *au, double *star_part, int it, double *scal, const double *rr_part, int nrr,
                const double *r_vec, hipStream_t st)
{
    if (g.lpc_row >= 64)
        row_gather_l<64>(g, c, a, v, au, star_part, it, scal, rr_part, nrr, r_vec, st);
    else if (g.lpc_row >= 32)
        row_gather_l<32>(g, c, a, v, au, star_part, it, scal, rr_part, nrr, r_vec, st);
    else if (g.lpc_row >= 16)
        row_gather_l<16>(g, c, a, v, au, star_part, it, scal, rr_part, nrr, r_vec, st);
    else
        row_gather_l<4>(g, c, a, v, au, star_part, it, scal, rr_part, nrr, r_vec, st);
}

template <int L, typename VT>
void row_gather_cg_lt(const GatherPlan &g, const CsrView &c, const double *a, CgState &s, int it,
                      hipStream_t st)
{
    hipLaunchKernelGGL((k_row_gather_cg<L, VT>), dim3(g.row_blocks), dim3(1024),
                       (size_t)c.n * sizeof(double), st, (int)c.m, (int)c.n, c.col,
                       (const VT *)c.val, c.len, c.istar, a, s.au, s.star_part, g.nstar,
                       g.star_chunk, it, s.scal, s.pap_part, g.col_blocks, s.x, s.r, s.r2, s.p,
                       s.Ap);
}

template <typename VT>
void row_gather_cg_t(const GatherPlan &g, const CsrView &c, const double *a, CgState &s, int it,
                     hipStream_t st)
{
    if (g.lpc_row >= 64)
        row_gather_cg_lt<64, VT>(g, c, a, s, it, st);
    else if (g.lpc_row >= 32)
        row_gather_cg_lt<32, VT>(g, c, a, s, it, st);
    else if (g.lpc_row >= 16)
        row_gather_cg_lt<16, VT>(g, c, a, s, it, st);
    else
        row_gather_cg_lt<4, VT>(g, c, a, s, it, st);
}

template <int L, typename VT>
void col_gather_lt(const GatherPlan &g, const CsrView &c, const double *a, const double *au,
                   const double *star_part, double *v, double eta, double shift, double *y, int it,
                   const double *scal, const double *r_vec, double *pap_part, hipStream_t st)
{
    const VT *val = (const VT *)c.val, *cval = (const VT *)c.cval;
    if (g.lds)
        hipLaunchKernelGGL((k_col_gather_lds<L, VT>), dim3(g.col_blocks), dim3(1024),
                           (size_t)c.m * sizeof(double), st, (int)c.m, (int)c.n, c.colptr,
                           c.rowidx, cval, au, c.d, val, c.istar, a, star_part, g.nstar, v,
                           eta, shift, y, it, scal, r_vec, pap_part);
    else
        hipLaunchKernelGGL((k_col_gather<L, VT>), dim3(g.col_blocks), dim3(256), 0, st, (int)c.n,
                           c.colptr, c.rowidx, cval, au, c.d, val, c.istar, a, star_part,
                           g.nstar, v, eta, shift, y, it, scal, r_vec, pap_part);
}

template <int L>
void col_gather_l(const GatherPlan &g, const CsrView &c, const double *a, const double *au,
                  const double *star_part, double *v, double eta, double shift, double *y, int it,
                  const double *scal, const double *r_vec, double *pap_part, hipStream_t st)
{
    if (c.f32)
        col_gather_lt<L, float>(g, c, a, au, star_part, v, eta, shift, y, it, scal, r_vec,
                                pap_part, st);
    else
        col_gather_lt<L, double>(g, c, a, au, star_part, v, eta, shift, y, it, scal, r_vec,
                                 pap_part, st);
}

void col_gather(const GatherPlan &g, const CsrView &c, const double *a, const double *au,
                const double *star_part, double *v, double eta, double shift, double *y, int it,
                const double *scal, const double *r_vec, double *pap_part, hipStream_t st)
{
    if (g.lpc_col >= 64)
        col_gather_l<64>(g, c, a, au, star_part, v, eta, shift, y, it, scal, r_vec, pap_part, st);
    else if (g.lpc_col >= 32)
        col_gather_l<32>(g, c, a, au, star_part, v, eta, shift, y, it, scal, r_vec, pap_part, st);
    else if (g.lpc_col >= 16)
        col_gather_l<16>(g, c, a, au, star_part, v, eta, shift, y, it, scal, r_vec, pap_part, st);
    else
        col_gather_l<4>(g, c, a, au, star_part, v, eta, shift, y, it, scal, r_vec, pap_part, st);
}
}  // namespace

hipError_t launch_hvp(const GatherPlan &g, const CsrView &c, const double *a, double eta,
                      double shift, const double *v, double *y, double *au, double *star_part,
                      hipStream_t st)
{
    row_gather(g, c, a, v, au, star_part, 0, nullptr, nullptr, 0, nullptr, st);
    col_gather(g, c, a, au, star_part, const_cast<double *>(v), eta, shift, y, 0, nullptr,
               nullptr, nullptr, st);
    return hipGetLastError();
}

hipError_t launch_cg_init(int64_t n, const double *rhs, double tol, int maxit, CgState &s,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(1024), 0, st, (int)n, rhs, tol, maxit, s.x, s.r,
                       s.p, s.scal);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(const GatherPlan &g, const CsrView &c, const double *a, double eta,
                               double shift, CgState &s, int it, hipStream_t st)
{
    if (g.fused) {
        // two kernels: the row gather also finishes iteration it-1's vector update
        if (c.f32)
            row_gather_cg_t<float>(g, c, a, s, it, st);
        else
            row_gather_cg_t<double>(g, c, a, s, it, st);
        col_gather(g, c, a, s.au, s.star_part, s.p, eta, shift, s.Ap, it, s.scal,
                   (it & 1) ? s.r2 : s.r, s.pap_part, st);
        return hipGetLastError();
    }
    // 1) p_new = r + beta p (beta, rr, done from the update partials); au = a.(P p_new)
    row_gather(g, c, a, s.p, s.au, s.star_part, it, s.scal, s.rr_part, g.upd_blocks, s.r, st);
    // 2) p = p_new; Ap; partials of p.Ap
    col_gather(g, c, a, s.au, s.star_part, s.p, eta, shift, s.Ap, it, s.scal, s.r, s.pap_part,
               st);
    // 3) alpha; x, r; partials of r.r
    hipLaunchKernelGGL(k_cg_update, dim3(g.upd_blocks), dim3(256), 0, st, (int)c.n, it, s.x, s.r,
                       s.p, s.Ap, s.scal, s.pap_part, g.col_blocks, s.rr_part);
    return hipGetLastError();
}

hipError_t launch_cg_check(const GatherPlan &g, CgState &s, int it, int64_t n, hipStream_t st)
{
    if (g.fused) {
        hipLaunchKernelGGL(k_cg_state, dim3(1), dim3(1024), 0, st, it, (int)n, s.scal,
                           s.pap_part, g.col_blocks, s.x, s.r, s.r2, s.p, s.Ap);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(256), 0, st, it, s.scal, s.rr_part, g.upd_blocks);
    return hipGetLastError();
}

hipError_t launch_make_w(const double *s, const double *gamma, double q, double eta, int64_t n,
                         int split, double *w, double *wlo, hipStream_t st)
{
    hipLaunchKernelGGL(k_make_w, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (int)n, s,
                       gamma, eta, q, split, w, wlo);
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

hipError_t launch_export_csr(int64_t m, int64_t n, const int32_t *col, const void *val, int f32,
                             const int32_t *len, int64_t *row_ptr, int32_t *ocol, double *oval,
                             int64_t cap, hipStream_t st)
{
    hipLaunchKernelGGL(k_scan32, dim3(1), dim3(1024), 0, st, (int)m, len, row_ptr);
    if (f32)
        hipLaunchKernelGGL((k_export_csr<float>), dim3((unsigned)m), dim3(256), 0, st, (int)m,
                           (int)n, col, (const float *)val, row_ptr, ocol, oval, cap);
    else
        hipLaunchKernelGGL((k_export_csr<double>), dim3((unsigned)m), dim3(256), 0, st, (int)m,
                           (int)n, col, (const double *)val, row_ptr, ocol, oval, cap);
    return hipGetLastError();
}

}  // namespace ibsn
