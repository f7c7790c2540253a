// dense_passes.hip -- the m x n streaming passes of the IBSN hot path on gfx950.
//
// Every pass reads the cost matrix once, row by row.  A workgroup owns a contiguous
// block of rows and holds one whole row in registers: thread t of NT owns the
// columns j = (q*NT + t)*VEC + v (q < Q, v < VEC), loaded as 16-byte vectors, so a
// row is Q coalesced sweeps of NT*16 bytes.  Because the row stays on chip, each
// pass needs one exp per entry: the row maximum / normaliser come from workgroup
// reductions (wave butterflies, then LDS across the waves) and the entries are
// then reused from registers.  Column sums (P^T a, d = P_rho^T a, the rounding sums)
// are accumulated per thread in registers over the workgroup's rows and written
// once as a partial row; a second kernel adds the partials in a fixed order, so no
// floating point atomics are used and results are run-to-run reproducible.
//
// The row after the current one is prefetched into a second register set while the
// current one is reduced, which keeps loads in flight across the reductions.
//
// Exponents.  Column potentials w_j and row shifts M_i both lie on a grid of spacing
// q (a power of two chosen per outer iteration), so w_j - M_i is exact and
//     x_ij = fma(-sigma, C_ij, w_j - M_i)
// is theta_ij - M_i with one rounding at the scale of x_ij, however large sigma and
// the potentials grow.  grid(v) = q * rint(v / q).
#include "ibsn_internal.h"
#include "solver_kernels.h"

#include <math.h>

namespace ibsn {
namespace {

constexpr int WAVE = 64;
enum { OP_SUM = 0, OP_MAX = 1, OP_MIN = 2 };

template <int OP>
__device__ __forceinline__ double comb(double x, double y)
{
    if constexpr (OP == OP_SUM)
        return x + y;
    else if constexpr (OP == OP_MAX)
        return fmax(x, y);
    else
        return fmin(x, y);
}

// Move a double across lanes with a DPP control (all 64 lanes active).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Wave reduction without LDS: within each row of 16 lanes, DPP lane ^ 1 and lane ^ 2
// (quad permutes), then rotations by 4 and 8; lane 16 r then holds row r's result, and
// the four rows are combined in a fixed order.  Every lane returns the same value.
// Call with all 64 lanes active.
template <int OP>
__device__ __forceinline__ double wave_red(double v)
{
    v = comb<OP>(v, dpp_mov<0xB1>(v));    // quad_perm [1,0,3,2]
    v = comb<OP>(v, dpp_mov<0x4E>(v));    // quad_perm [2,3,0,1]
    v = comb<OP>(v, dpp_mov<0x124>(v));   // row_ror:4
    v = comb<OP>(v, dpp_mov<0x128>(v));   // row_ror:8
    return comb<OP>(comb<OP>(readlane_d(v, 0), readlane_d(v, 16)),
                    comb<OP>(readlane_d(v, 32), readlane_d(v, 48)));
}

// Workgroup reduction of K values with per-slot operators.  `lds` holds two buffers of
// K*(NT/64) doubles used alternately, so one barrier per reduction suffices: a buffer
// is rewritten only after every wave has passed the barrier of the next reduction.
template <int NT, int... OPS>
struct BlockRed {
    static constexpr int K = sizeof...(OPS);
    static constexpr int NW = NT / WAVE;
    static constexpr int LDS = 2 * K * NW;

    template <int I, int OP, int... REST>
    __device__ __forceinline__ static void wave_all(double *v)
    {
        v[I] = wave_red<OP>(v[I]);
        if constexpr (sizeof...(REST) > 0)
            wave_all<I + 1, REST...>(v);
    }
    template <int I, int OP, int... REST>
    __device__ __forceinline__ static void fold_all(double *v, const double *buf)
    {
        double r = buf[I * NW];
#pragma unroll
        for (int k = 1; k < NW; ++k)
            r = comb<OP>(r, buf[I * NW + k]);
        v[I] = r;
        if constexpr (sizeof...(REST) > 0)
            fold_all<I + 1, REST...>(v, buf);
    }
    __device__ __forceinline__ static void run(double *v, double *lds, int &parity)
    {
        double *buf = lds + parity * K * NW;
        parity ^= 1;
        wave_all<0, OPS...>(v);
        const int w = threadIdx.x / WAVE;
        if ((threadIdx.x & (WAVE - 1)) == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                buf[k * NW + w] = v[k];
        }
        __syncthreads();
        fold_all<0, OPS...>(v, buf);
    }
};

template <typename CT, int VEC>
struct VecLoad;
template <>
struct VecLoad<double, 2> {
    __device__ __forceinline__ static void get(const double *p, double *x)
    {
        const double2 v = *reinterpret_cast<const double2 *>(p);
        x[0] = v.x;
        x[1] = v.y;
    }
};
template <>
struct VecLoad<float, 4> {
    __device__ __forceinline__ static void get(const float *p, float *x)
    {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        x[0] = v.x;
        x[1] = v.y;
        x[2] = v.z;
        x[3] = v.w;
    }
};

template <int NT, int VEC>
__device__ __forceinline__ int col_of(int e)
{
    return ((e / VEC) * NT + (int)threadIdx.x) * VEC + (e % VEC);
}

// Load row `row` (n entries) into x[Q*VEC] (cost type) without branches per slot.
// When the row starts on a 16-byte boundary and n is a multiple of VEC, every slot is a
// 16-byte vector load whose start is clamped to the last full vector of the row;
// otherwise scalar loads with each column clamped to n - 1.  Either way every address is
// inside the row, and slots past n hold copies of in-row values: every caller masks
// those slots (col_of(e) >= n) before their values are used.
template <int NT, int Q, int QF, int VEC, bool VECOK, typename CT>
__device__ __forceinline__ void load_row(const CT *__restrict__ row, int n, CT *x)
{
    if constexpr (VECOK) {
        // every row starts on a 16-byte boundary and n % VEC == 0 (checked per launch),
        // so each slot start, a multiple of VEC, is 16-byte aligned
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int j0 = (q * NT + (int)threadIdx.x) * VEC;
            const CT *p = static_cast<const CT *>(
                __builtin_assume_aligned(row + (q < QF ? j0 : min(j0, n - VEC)), 16));
            VecLoad<CT, VEC>::get(p, x + q * VEC);
        }
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int j0 = (q * NT + (int)threadIdx.x) * VEC;
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                x[q * VEC + v] = row[q < QF ? j0 + v : min(j0 + v, n - 1)];
        }
    }
}

template <int NT, int Q, int VEC>
__device__ __forceinline__ void store_cols(double *__restrict__ dst, int n, const double *x)
{
#pragma unroll
    for (int e = 0; e < Q * VEC; ++e) {
        const int j = col_of<NT, VEC>(e);
        if (j < n)
            dst[j] = x[e];
    }
}

// Copy an n-vector into this workgroup's dynamic LDS (one value per column).
__device__ __forceinline__ void stage_lds(const double *__restrict__ src, int n, double *lds)
{
    for (int j = threadIdx.x; j < n; j += blockDim.x)
        lds[j] = src[j];
    __syncthreads();
}

__device__ __forceinline__ double grid(double v, double q) { return q * rint(v / q); }

// exp(x) for finite x <= 709, by table-driven argument reduction (P. T. P. Tang,
// "Table-driven implementation of the exponential function in IEEE floating-point
// arithmetic", ACM TOMS 15(2), 1989): x = (128 e + j) ln2/128 + r with |r| <= ln2/256, so
// exp(x) = 2^e 2^(j/128) exp(r), and exp(r) - 1 is its Taylor polynomial of degree 5
// (the next term is below 6e-19 relative).
//  - k = round(x 128/ln2) comes from one fused multiply-add with 1.5*2^52, whose unit in
//    the last place is 1: the sum holds k in the low word of its bit pattern.
//  - ln2/128 is split into a double and its remainder; with fused multiply-adds the
//    reduced argument is exact to the last bit of r.
//  - x <= -746 gives 0 (clamped; the result underflows); NaN also gives 0, so the
//    callers require finite costs and potentials.
// etab[j] = 2^(j/128), see exp_table_init.  The passes never produce x > 709: x is
// theta - M_i with M_i the grid-rounded row maximum.
constexpr int EXP_TAB = 128;
constexpr double EXP_SHIFT = 0x1.8p52;               // 1.5 * 2^52
constexpr double EXP_INV_L = 0x1.71547652b82fep+7;   // 128 / ln 2
constexpr double EXP_L_HI = 0x1.62e42fefa39efp-8;    // ln 2 / 128, rounded
constexpr double EXP_L_LO = 0x1.abc9e3b39803fp-63;   // ln 2 / 128 - EXP_L_HI

__device__ __forceinline__ double exp_tab(double x, const double *__restrict__ etab)
{
    x = fmax(x, -746.0);
    const double t = fma(x, EXP_INV_L, EXP_SHIFT);
    const int k = __double2loint(t);
    const double kd = t - EXP_SHIFT;
    double r = fma(-kd, EXP_L_HI, x);
    r = fma(-kd, EXP_L_LO, r);
    double p = fma(r, 1.0 / 120.0, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p *= r;                                   // exp(r) - 1
    const double tj = etab[k & (EXP_TAB - 1)];
    return ldexp(fma(tj, p, tj), k >> 7);
}

// 2^(j/128), j < 128, into LDS (one barrier)
__device__ __forceinline__ void exp_table_init(double *etab)
{
    for (int j = threadIdx.x; j < EXP_TAB; j += blockDim.x)
        etab[j] = exp2((double)j * (1.0 / EXP_TAB));
    __syncthreads();
}

// Slot e of a thread holds column col_of(e).  The tiles are chosen so that the first QF
// slabs (slots e < QF*VEC) lie inside the row for every thread; only later slabs can
// reach past n and need a mask.
template <int QF, int NT, int VEC>
__device__ __forceinline__ bool slot_valid(int e, int n)
{
    return e / VEC < QF || col_of<NT, VEC>(e) < n;
}

// column of slot e, clamped into [0, n) in the slabs that may reach past n
template <int QF, int NT, int VEC>
__device__ __forceinline__ int slot_col(int e, int n)
{
    const int j = col_of<NT, VEC>(e);
    return e / VEC < QF ? j : min(j, n - 1);
}

// w at the owned columns; padding slots get -inf so that exp of their argument is 0
template <int NT, int Q, int VEC>
__device__ __forceinline__ void load_w(const double *__restrict__ w, int n, double *x)
{
#pragma unroll
    for (int e = 0; e < Q * VEC; ++e) {
        const int j = col_of<NT, VEC>(e);
        x[e] = j < n ? w[j] : -INFINITY;
    }
}

__device__ __forceinline__ void row_range(int m, int &i0, int &i1)
{
    const int64_t g = blockIdx.x, G = gridDim.x;
    i0 = (int)((int64_t)m * g / G);
    i1 = (int)((int64_t)m * (g + 1) / G);
}

// Per-row scalars (shifts, normalisers, weights) are staged in LDS ROWCH rows at a time,
// so that the row loop reads them from LDS instead of waiting on memory every row.
constexpr int ROWCH = 64;

// Row loop of a workgroup over its rows [i0, i1).  Row i+1 is loaded into a second
// register set while row i is processed, so its loads are in flight across the whole of
// the current row.  stage(i) runs before rows i .. i+ROWCH-1 are touched (it fills the
// LDS row scalars; it begins and ends with a barrier); body(i, slot, x) processes row i
// held in x, with slot = its index in the staged chunk.
template <int NT, int Q, int QF, int VEC, bool VECOK, bool PREFETCH, typename CT,
          typename Stage, typename Body>
__device__ __forceinline__ void row_loop_v(const CT *__restrict__ C, int64_t ldc, int n, int i0,
                                           int i1, Stage &stage, Body &body)
{
    CT xr[Q * VEC];
    if constexpr (PREFETCH) {
        CT xn[Q * VEC];
        if (i0 < i1)
            load_row<NT, Q, QF, VEC, VECOK>(C + (int64_t)i0 * ldc, n, xr);
        for (int i = i0; i < i1; ++i) {
            const int slot = (i - i0) & (ROWCH - 1);
            if (slot == 0)
                stage(i);
            if (i + 1 < i1)
                load_row<NT, Q, QF, VEC, VECOK>(C + (int64_t)(i + 1) * ldc, n, xn);
            body(i, slot, xr);
#pragma unroll
            for (int e = 0; e < Q * VEC; ++e)
                xr[e] = xn[e];
        }
    } else {
        for (int i = i0; i < i1; ++i) {
            const int slot = (i - i0) & (ROWCH - 1);
            if (slot == 0)
                stage(i);
            load_row<NT, Q, QF, VEC, VECOK>(C + (int64_t)i * ldc, n, xr);
            body(i, slot, xr);
        }
    }
}

// 16-byte vector loads when the matrix start and the row pitch are 16-byte aligned and n
// is a multiple of VEC (the same for every row); scalar loads otherwise.
// PREFETCH = false (passes whose per-entry state leaves no registers for a second row):
// each row is loaded when it is reached.
template <int NT, int Q, int QF, int VEC, bool PREFETCH = true, typename CT, typename Stage,
          typename Body>
__device__ __forceinline__ void row_loop(const CT *__restrict__ C, int64_t ldc, int n, int i0,
                                         int i1, Stage &&stage, Body &&body)
{
    const bool vec_ok = (reinterpret_cast<uintptr_t>(C) & 15u) == 0 &&
                        ((uint64_t)ldc * sizeof(CT)) % 16 == 0 && n % VEC == 0;
    if (vec_ok)
        row_loop_v<NT, Q, QF, VEC, true, PREFETCH>(C, ldc, n, i0, i1, stage, body);
    else
        row_loop_v<NT, Q, QF, VEC, false, PREFETCH>(C, ldc, n, i0, i1, stage, body);
}

// Copy rows [i, min(i + ROWCH, i1)) of up to four m-vectors into LDS (null: skipped).
__device__ __forceinline__ void stage_rows(int i, int i1, const double *__restrict__ s0,
                                           double *d0, const double *__restrict__ s1, double *d1,
                                           const double *__restrict__ s2, double *d2,
                                           const double *__restrict__ s3 = nullptr,
                                           double *d3 = nullptr)
{
    __syncthreads();   // the previous chunk may still be read
    const int cnt = min(ROWCH, i1 - i);
    for (int r = threadIdx.x; r < cnt; r += blockDim.x) {
        if (s0)
            d0[r] = s0[i + r];
        if (s1)
            d1[r] = s1[i + r];
        if (s2)
            d2[r] = s2[i + r];
        if (s3)
            d3[r] = s3[i + r];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------------
// eval: M_i = max_j theta_ij, S_i = sum_j exp(theta_ij - M_i), column partials of
// a_i P_ij, objective row terms a_i ((r_i + M_i) + log S_i).
// ---------------------------------------------------------------------------------
template <int NT, int Q, int QF, int VEC, typename CT>
__global__ __launch_bounds__(NT) void k_eval(const CT *__restrict__ C, int64_t ldc, int m, int n,
                                             double sigma, double qg,
                                             const double *__restrict__ w,
                                             const double *__restrict__ a,
                                             const double *__restrict__ r, double *__restrict__ Mo,
                                             double *__restrict__ So, double *__restrict__ lse,
                                             double *__restrict__ plan,
                                             double *__restrict__ colpart,
                                             double *__restrict__ rowpart)
{
    constexpr int E = Q * VEC;
    constexpr int NW = NT / WAVE;
    // per row: each wave takes its own shift m_w = grid(wave max of theta) and sums
    // exp(theta - m_w); one barrier publishes the (m_w, s_w) pairs; every wave then forms
    // M = max_w m_w = grid(max theta) (grid rounding is monotone) and
    // S = sum_w s_w exp(m_w - M), and scales its entries by exp(m_w - M).  All shifts
    // lie on the grid, so m_w - M is exact.  The pair buffer alternates between rows.
    __shared__ double pairs[2][2 * NW];
    __shared__ double etab[EXP_TAB];
    extern __shared__ double wl[];   // w staged in LDS (n doubles)
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    exp_table_init(etab);
    stage_lds(w, n, wl);
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    __shared__ double rA[ROWCH], rR[ROWCH];
    double acc[E], x[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        acc[e] = 0.0;
    double rowacc = 0.0;
    row_loop<NT, Q, QF, VEC>(
        C, ldc, n, i0, i1, [&](int i) { stage_rows(i, i1, a, rA, r, rR, nullptr, nullptr); },
        [&](int i, int slot, const CT *xr) {
        // padding slots: theta = -inf, so they drop out of the max and p = 0; a wave
        // with no column in the row gets m_w = -inf, s_w = 0 and factor 0
        double mt = -INFINITY;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double th = fma(-sigma, (double)xr[e], wl[slot_col<QF, NT, VEC>(e, n)]);
            mt = fmax(mt, slot_valid<QF, NT, VEC>(e, n) ? th : -INFINITY);
        }
        const double mw = grid(wave_red<OP_MAX>(mt), qg);
        double st = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double xa = fma(-sigma, (double)xr[e], wl[slot_col<QF, NT, VEC>(e, n)] - mw);
            const double p = exp_tab(slot_valid<QF, NT, VEC>(e, n) ? xa : -INFINITY, etab);
            x[e] = p;
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
        const double mk = lane < NW ? pr[lane] : -INFINITY;
        const double M = wave_red<OP_MAX>(mk);
        const double term = lane < NW ? pr[NW + lane] * exp_tab(mk - M, etab) : 0.0;
        const double S = wave_red<OP_SUM>(term);
        const double ai = rA[slot];
        const double sc = ai / S * exp_tab(mw - M, etab);   // a_i exp(m_w - M) / S
#pragma unroll
        for (int e = 0; e < E; ++e)
            acc[e] = fma(sc, x[e], acc[e]);
        if (plan) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = col_of<NT, VEC>(e);
                if (j < n)
                    plan[(int64_t)i * n + j] = sc * x[e];
            }
        }
        if (threadIdx.x == 0) {
            const double ls = log(S);
            Mo[i] = M;
            So[i] = S;
            if (lse)
                lse[i] = M + ls;
            if (r)
                rowacc += ai * ((rR[slot] + M) + ls);
        }
        });
    store_cols<NT, Q, VEC>(colpart + (int64_t)blockIdx.x * n, n, acc);
    if (threadIdx.x == 0)
        rowpart[blockIdx.x] = rowacc;
}

// ---------------------------------------------------------------------------------
// Armijo trial from the row state M of the base point, tau = t*Delta/eta:
//   q = exp(theta - M_i), A = sum q, small step (BIG=0, cv = expm1(tau)):
//   B = sum q*cv, qe = q + q*cv = q e^tau, delta = log1p(B/A);
//   big step (BIG=1, cv = exp(tau - tau_shift)): qe = q*cv, delta = tau_shift + log(Z/A).
//   Z = sum qe, P'_ij = qe / Z, new state M' = M + tau_shift + log(max qe), S' = Z / max qe.
// ---------------------------------------------------------------------------------
template <int NT, int Q, int QF, int VEC, typename CT, int BIG>
__global__ __launch_bounds__(NT) void k_trial(const CT *__restrict__ C, int64_t ldc, int m, int n,
                                              double sigma, double qg,
                                              const double *__restrict__ w,
                                              const double *__restrict__ a,
                                              const double *__restrict__ Mb,
                                              const double *__restrict__ colv,
                                              const double *__restrict__ scal,
                                              double *__restrict__ Mn, double *__restrict__ Sn,
                                              double *__restrict__ colpart,
                                              double *__restrict__ rowpart)
{
    constexpr int E = Q * VEC;
    using Red = BlockRed<NT, OP_SUM, OP_SUM, OP_SUM, OP_MAX>;
    __shared__ double lds[Red::LDS];
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    if ((scal[SC_BIG] != 0.0) != (BIG != 0))
        return;   // the other form of the trial handles this step
    const double tau_shift = scal[SC_TAUSHIFT];
    extern __shared__ double cvl[];   // colv staged in LDS (n doubles)
    __shared__ double etab[EXP_TAB];
    __shared__ double rM[ROWCH], rA[ROWCH];
    double wr[E], acc[E], x[E];
    exp_table_init(etab);
    load_w<NT, Q, VEC>(w, n, wr);   // padding slots: -inf, so q = 0 there
    stage_lds(colv, n, cvl);
#pragma unroll
    for (int e = 0; e < E; ++e)
        acc[e] = 0.0;
    double rowacc = 0.0;
    row_loop<NT, Q, QF, VEC>(
        C, ldc, n, i0, i1,
        [&](int i) { stage_rows(i, i1, Mb, rM, a, rA, nullptr, nullptr); },
        [&](int i, int slot, const CT *xr) {
        const double Mi = rM[slot];
        double red[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double q = exp_tab(fma(-sigma, (double)xr[e], wr[e] - Mi), etab);
            const double cv = cvl[slot_col<QF, NT, VEC>(e, n)];   // finite, and q = 0 on padding
            red[0] += q;
            double qe;
            if constexpr (BIG) {
                qe = q * cv;
            } else {
                const double qf = q * cv;
                red[1] += qf;
                qe = q + qf;
            }
            red[2] += qe;
            red[3] = fmax(red[3], qe);
            x[e] = qe;
        }
        Red::run(red, lds, parity);
        const double A = red[0], B = red[1], Z = red[2], mx = red[3];
        const double ai = rA[slot];
        const double sc = ai / Z;
#pragma unroll
        for (int e = 0; e < E; ++e)
            acc[e] = fma(sc, x[e], acc[e]);
        if (threadIdx.x == 0) {
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
    store_cols<NT, Q, VEC>(colpart + (int64_t)blockIdx.x * n, n, acc);
    if (threadIdx.x == 0)
        rowpart[blockIdx.x] = rowacc;
}

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

// ---------------------------------------------------------------------------------
// Stop test pass 1 (Algorithm 3, steps 2-8): X = a_i P; z_i; column sums of X and z X.
// ---------------------------------------------------------------------------------
template <int NT, int Q, int QF, int VEC, typename CT>
__global__ __launch_bounds__(NT) void k_stop1(const CT *__restrict__ C, int64_t ldc, int m, int n,
                                              double sigma, const double *__restrict__ w,
                                              const double *__restrict__ a,
                                              const double *__restrict__ M,
                                              const double *__restrict__ S,
                                              double *__restrict__ z, double *__restrict__ colpart,
                                              double *__restrict__ colpart2,
                                              double *__restrict__ rowpart)
{
    constexpr int E = Q * VEC;
    using RedSum = BlockRed<NT, OP_SUM>;
    __shared__ double lds[RedSum::LDS];
    __shared__ double rM[ROWCH], rS[ROWCH], rA[ROWCH];
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    extern __shared__ double wl[];   // w staged in LDS (n doubles)
    __shared__ double etab[EXP_TAB];
    double ax[E], az[E], x[E];
    exp_table_init(etab);
    stage_lds(w, n, wl);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        ax[e] = 0.0;
        az[e] = 0.0;
    }
    double rowacc = 0.0;
    row_loop<NT, Q, QF, VEC>(
        C, ldc, n, i0, i1, [&](int i) { stage_rows(i, i1, M, rM, S, rS, a, rA); },
        [&](int i, int slot, const CT *xr) {
            const double Mi = rM[slot], ai = rA[slot], aS = ai / rS[slot];
            double red[1] = {0.0};
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const bool valid = slot_valid<QF, NT, VEC>(e, n);
                const double xa =
                    fma(-sigma, (double)xr[e], wl[slot_col<QF, NT, VEC>(e, n)] - Mi);
                const double X = exp_tab(valid ? xa : -INFINITY, etab) * aS;
                x[e] = X;
                red[0] += X;
            }
            RedSum::run(red, lds, parity);
            const double rs = red[0];
            const double zi = fmin(ai / rs, 1.0);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                ax[e] += x[e];
                az[e] = fma(zi, x[e], az[e]);
            }
            if (threadIdx.x == 0) {
                z[i] = zi;
                rowacc += (rs - ai) * (rs - ai);
            }
        });
    store_cols<NT, Q, VEC>(colpart + (int64_t)blockIdx.x * n, n, ax);
    store_cols<NT, Q, VEC>(colpart2 + (int64_t)blockIdx.x * n, n, az);
    if (threadIdx.x == 0)
        rowpart[blockIdx.x] = rowacc;
}

// ---------------------------------------------------------------------------------
// Stop test pass 2: e_r (row-local), Xhat = z X y + e_r e_c^T / ||e_r||_1 (Algorithm 3,
// steps 9-11), D_phi(Xhat, X) in the log domain, <C,Xhat>, <C,X>, c-transforms of
// gamma and psi, <X, U(gamma, zeta^c)>, norms for Delta_kkt.
// ---------------------------------------------------------------------------------
template <int NT, int Q, int QF, int VEC, typename CT>
__global__ __launch_bounds__(NT) void k_stop2(const CT *__restrict__ C, int64_t ldc, int m, int n,
                                              double sigma, const double *__restrict__ w,
                                              const double *__restrict__ a,
                                              const double *__restrict__ M,
                                              const double *__restrict__ S,
                                              const double *__restrict__ gamma,
                                              const double *__restrict__ psi,
                                              const double *__restrict__ y,
                                              const double *__restrict__ ec,
                                              const double *__restrict__ z, double er1,
                                              double *__restrict__ xhat,
                                              double *__restrict__ rowpart)
{
    constexpr int E = Q * VEC;
    using Red3 = BlockRed<NT, OP_SUM, OP_MIN, OP_MIN>;
    using RedEnd = BlockRed<NT, OP_SUM, OP_SUM, OP_SUM, OP_SUM, OP_MIN, OP_SUM, OP_SUM>;
    __shared__ double lds[Red3::LDS + RedEnd::LDS];
    extern __shared__ double wl[];   // w staged in LDS (n doubles)
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    __shared__ double etab[EXP_TAB];
    exp_table_init(etab);
    stage_lds(w, n, wl);
    __shared__ double rM[ROWCH], rS[ROWCH], rA[ROWCH], rZ[ROWCH];
    double X[E];
    double t_dphi = 0.0, t_cxh = 0.0, t_cx = 0.0, t_xu = 0.0, t_xhmin = INFINITY, t_xf = 0.0,
           t_cf = 0.0;
    double azg = 0.0, azp = 0.0;
    const double inv_er1 = er1 > 0.0 ? 1.0 / er1 : 0.0;
    row_loop<NT, Q, QF, VEC, false>(
        C, ldc, n, i0, i1, [&](int i) { stage_rows(i, i1, M, rM, S, rS, a, rA, z, rZ); },
        [&](int i, int slot, const CT *cst) {
        const double Mi = rM[slot], ai = rA[slot], zi = rZ[slot], aS = ai / rS[slot];
        double red[3] = {0.0, INFINITY, INFINITY};
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool valid = slot_valid<QF, NT, VEC>(e, n);
            const int j = slot_col<QF, NT, VEC>(e, n);
            const double c = valid ? (double)cst[e] : 0.0;
            const double Xv = exp_tab(valid ? fma(-sigma, c, wl[j] - Mi) : -INFINITY, etab) * aS;
            X[e] = Xv;
            red[0] = fma(Xv, y[j], red[0]);
            red[1] = fmin(red[1], valid ? c - gamma[j] : INFINITY);
            red[2] = fmin(red[2], valid ? c - psi[j] : INFINITY);
        }
        Red3::run(red, lds, parity);
        const double eri = fmax(ai - zi * red[0], 0.0);   // >= 0 exactly; clamp rounding
        const double zg = red[1], zp = red[2];
        const double lr = log(ai) - log(rS[slot]);   // log X_ij = lr + (theta_ij - M_i)
        const double es = eri * inv_er1;         // rank-one factor e_r,i / ||e_r||_1
#pragma unroll 2
        for (int e = 0; e < E; ++e) {
            const bool valid = slot_valid<QF, NT, VEC>(e, n);
            const int j = slot_col<QF, NT, VEC>(e, n);
            const double c = valid ? (double)cst[e] : 0.0;
            const double Xv = X[e];
            const double f = (zi * Xv) * y[j];
            const double xh = valid ? fma(es, ec[j], f) : 0.0;
            const double lx = lr + fma(-sigma, c, wl[j] - Mi);
            const bool pos = xh > 0.0;
            const double lxh = log(pos ? xh : 1.0);
            t_dphi += pos ? (xh * (lxh - lx) - xh) + Xv : Xv;
            t_cxh = fma(c, xh, t_cxh);
            t_cx = fma(c, Xv, t_cx);
            t_xhmin = fmin(t_xhmin, valid ? xh : INFINITY);
            t_xu = fma(Xv, (c - gamma[j]) - zg, t_xu);
            t_xf = fma(Xv, Xv, t_xf);
            t_cf = fma(c, c, t_cf);
            if (xhat && valid)
                xhat[(int64_t)i * n + col_of<NT, VEC>(e)] = xh;
        }
        if (threadIdx.x == 0) {
            azg += ai * zg;
            azp += ai * zp;
        }
        });
    double fin[7] = {t_dphi, t_cxh, t_cx, t_xu, t_xhmin, t_xf, t_cf};
    int p2 = 0;
    RedEnd::run(fin, lds + Red3::LDS, p2);
    if (threadIdx.x == 0) {
        double *o = rowpart + (int64_t)blockIdx.x * STOP2_NSLOT;
        o[STOP2_DPHI] = fin[0];
        o[STOP2_CXH] = fin[1];
        o[STOP2_AZG] = azg;
        o[STOP2_AZP] = azp;
        o[STOP2_CX] = fin[2];
        o[STOP2_XU] = fin[3];
        o[STOP2_XHMIN] = fin[4];
        o[STOP2_XF] = fin[5];
        o[STOP2_CF] = fin[6];
        o[STOP2_NEG] = 0.0;
    }
}

// ---------------------------------------------------------------------------------
// column reduction: out_j = sum_g part[g][j], g ascending within each of NW strided
// subsets, subsets added in order.  64 columns per workgroup.
// ---------------------------------------------------------------------------------
template <int NW>
__global__ __launch_bounds__(NW *WAVE) void k_colreduce(const double *__restrict__ part, int G, int n,
                                                        double *__restrict__ out,
                                                        const double *__restrict__ sub,
                                                        double *__restrict__ out2)
{
    __shared__ double s[NW][WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int j = blockIdx.x * WAVE + lane;
    double acc = 0.0;
    if (j < n)
        for (int g = wv; g < G; g += NW)
            acc += part[(int64_t)g * n + j];
    s[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && j < n) {
        double t = s[0][lane];
        for (int k = 1; k < NW; ++k)
            t += s[k][lane];
        out[j] = t;
        if (sub)
            out2[j] = t - sub[j];
    }
}

}  // namespace

// ---------------------------------------------------------------------------------
// host side: tile choice and launchers
// ---------------------------------------------------------------------------------
// Tiles (NT threads, Q vector slots per thread, QF slabs always inside the row).  Each
// tile serves n in (previous capacity, NT*Q*VEC], so the first QF slabs are full for
// every n it is chosen for.  Light tiles serve eval and stop pass 1; the heavy tile of the
// same row serves trial, sparsify and stop pass 2, which keep more values live per
// entry; both run on the same grid.  1024-thread tiles keep 10 entries per thread at
// n <= 10240 (FP64), which leaves room for four waves per SIMD.
struct TileRow {
    int cap;                  // largest n served
    int nt, q, qf;            // light tile
    int nt_h, q_h, qf_h;      // heavy tile
    int per_cu;               // workgroups per CU
};
const TileRow TILES64[] = {
    {512, 256, 1, 0, 256, 1, 0, 4},      {1024, 256, 2, 1, 256, 2, 1, 4},
    {1536, 256, 3, 2, 256, 3, 2, 4},     {2048, 256, 4, 3, 256, 4, 3, 4},
    {3072, 512, 3, 2, 512, 3, 2, 2},     {4096, 512, 4, 3, 512, 4, 3, 2},
    {6144, 1024, 3, 2, 512, 6, 4, 1},    {8192, 1024, 4, 3, 512, 8, 6, 1},
    {10240, 1024, 5, 4, 512, 10, 8, 1},
};
const TileRow TILES32[] = {
    {1024, 256, 1, 0, 256, 1, 0, 4},     {2048, 256, 2, 1, 256, 2, 1, 4},
    {3072, 256, 3, 2, 256, 3, 2, 4},     {4096, 256, 4, 3, 256, 4, 3, 4},
    {6144, 512, 3, 2, 512, 3, 2, 2},     {8192, 512, 4, 3, 512, 4, 3, 2},
    {12288, 1024, 3, 2, 512, 6, 4, 1},   {16384, 1024, 4, 3, 512, 8, 6, 1},
    {20480, 512, 10, 8, 512, 10, 8, 1},
};
#define IBSN_LIGHT_TILES(X) \
    X(256, 1, 0)            \
    X(256, 2, 1)            \
    X(256, 3, 2)            \
    X(256, 4, 3)            \
    X(512, 3, 2)            \
    X(512, 4, 3)            \
    X(1024, 3, 2)           \
    X(1024, 4, 3)           \
    X(1024, 5, 4)           \
    X(512, 10, 8)
#define IBSN_HEAVY_TILES(X) \
    X(256, 1, 0)            \
    X(256, 2, 1)            \
    X(256, 3, 2)            \
    X(256, 4, 3)            \
    X(512, 3, 2)            \
    X(512, 4, 3)            \
    X(512, 6, 4)            \
    X(512, 8, 6)            \
    X(512, 10, 8)

bool plan_rows(int64_t m, int64_t n, int cost_kind, int num_cus, RowPlan *p)
{
    const TileRow *t = cost_kind == 1 ? TILES32 : TILES64;
    const int nt = (int)(sizeof(TILES64) / sizeof(TILES64[0]));
    for (int k = 0; k < nt; ++k) {
        if (n <= t[k].cap) {
            p->nt = t[k].nt;
            p->q = t[k].q;
            p->qf = t[k].qf;
            p->nt_h = t[k].nt_h;
            p->q_h = t[k].q_h;
            p->qf_h = t[k].qf_h;
            p->vec = cost_kind == 1 ? 4 : 2;
            const int64_t g = (int64_t)num_cus * t[k].per_cu;
            p->grid = (int)(g < m ? g : m);
            return true;
        }
    }
    return false;
}

RowPlan heavy_plan(const RowPlan &p)
{
    RowPlan h = p;
    h.nt = p.nt_h;
    h.q = p.q_h;
    h.qf = p.qf_h;
    return h;
}

#define IBSN_DISPATCH(NT_, Q_, QF_, BODY)                                         \
    if (p.nt == NT_ && p.q == Q_ && p.qf == QF_) {                               \
        constexpr int NT = NT_, Q = Q_, QF = QF_;                                \
        if (d.cost_kind == 0) {                                                  \
            constexpr int VEC = 2;                                               \
            using CT = double;                                                   \
            BODY;                                                                \
        } else {                                                                 \
            constexpr int VEC = 4;                                               \
            using CT = float;                                                    \
            BODY;                                                                \
        }                                                                        \
        return hipGetLastError();                                                \
    }

hipError_t launch_eval(const RowPlan &p, const DenseArgs &d, const double *r, double *M, double *S,
                       double *lse, double *plan, double *colpart, double *rowpart, hipStream_t st)
{
#define BODY                                                                                     \
    hipLaunchKernelGGL((k_eval<NT, Q, QF, VEC, CT>), dim3(p.grid), dim3(NT),                         \
                       (size_t)d.n * sizeof(double), st,                                         \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.q, d.w, d.a, r, M, S, \
                       lse,                                                                      \
                       plan, colpart, rowpart)
#define X(a, b, c) IBSN_DISPATCH(a, b, c, BODY)
    IBSN_LIGHT_TILES(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

hipError_t launch_trial(const RowPlan &p_in, const DenseArgs &d, const double *M, const double *colv,
                        const double *scal, double *M_new, double *S_new, double *colpart,
                        double *rowpart, hipStream_t st)
{
    const RowPlan p = heavy_plan(p_in);
    const size_t lds_bytes = (size_t)d.n * sizeof(double);
#define BODY                                                                                      \
    hipLaunchKernelGGL((k_trial<NT, Q, QF, VEC, CT, 0>), dim3(p.grid), dim3(NT), lds_bytes, st,       \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.q, d.w, d.a, M, colv, \
                       scal, M_new, S_new, colpart, rowpart);                                     \
    hipLaunchKernelGGL((k_trial<NT, Q, QF, VEC, CT, 1>), dim3(p.grid), dim3(NT), lds_bytes, st,       \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.q, d.w, d.a, M, colv, \
                       scal, M_new, S_new, colpart, rowpart)
#define X(a, b, c) IBSN_DISPATCH(a, b, c, BODY)
    IBSN_HEAVY_TILES(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

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

hipError_t launch_stop1(const RowPlan &p, const DenseArgs &d, const double *M, const double *S,
                        double *z, double *colpart, double *colpart2, double *rowpart,
                        hipStream_t st)
{
    const size_t lds_bytes = (size_t)d.n * sizeof(double);
#define BODY                                                                                     \
    hipLaunchKernelGGL((k_stop1<NT, Q, QF, VEC, CT>), dim3(p.grid), dim3(NT), lds_bytes, st,                 \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.w, d.a, M, S, z,   \
                       colpart, colpart2, rowpart)
#define X(a, b, c) IBSN_DISPATCH(a, b, c, BODY)
    IBSN_LIGHT_TILES(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

hipError_t launch_stop2(const RowPlan &p_in, const DenseArgs &d, const double *M, const double *S,
                        const Stop2Vec &v, double *xhat, double *rowpart, hipStream_t st)
{
    const RowPlan p = heavy_plan(p_in);
    const size_t lds_bytes = (size_t)d.n * sizeof(double);
#define BODY                                                                                      \
    hipLaunchKernelGGL((k_stop2<NT, Q, QF, VEC, CT>), dim3(p.grid), dim3(NT), lds_bytes, st,                  \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.w, d.a, M, S,       \
                       v.gamma, v.psi, v.y, v.ec, v.z, v.er1, xhat, rowpart)
#define X(a, b, c) IBSN_DISPATCH(a, b, c, BODY)
    IBSN_HEAVY_TILES(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

hipError_t launch_colreduce(const double *part, int G, int64_t n, double *out, const double *sub,
                            double *out2, hipStream_t st)
{
    const int blocks = (int)((n + WAVE - 1) / WAVE);
    hipLaunchKernelGGL((k_colreduce<16>), dim3(blocks), dim3(16 * WAVE), 0, st, part, G, (int)n,
                       out, sub, out2);
    return hipGetLastError();
}

}  // namespace ibsn
