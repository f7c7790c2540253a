// dense_common.h -- shared device helpers and tile tables of the m x n streaming passes of the
// IBSN hot path on gfx950 (dense_eval.hip, dense_trial.hip, dense_sparsify.hip, dense_stop.hip).
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
// Exponents.  Column potentials are held in two parts, w_j = wh_j + wl_j: wh_j and the
// row shifts M_i lie on a grid of spacing q (a power of two chosen per outer iteration),
// so wh_j - M_i is exact, and wl_j is the small remainder (|wl_j| <= q/2).  Then
//     x_ij = fma(-sigma, C_ij, wh_j - M_i) + wl_j
// is theta_ij - M_i with two roundings at the scale of x_ij, however large sigma and the
// potentials grow, and the potentials themselves are not limited to the grid.
// grid(v) = q * rint(v / q).
#pragma once

#include "ibsn_internal.h"
#include "solver_kernels.h"

#include <math.h>

#include <atomic>
#include <type_traits>

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

// Move a double across lanes with a DPP control whose every lane has a source lane
// (quad permutes, row rotations, mirrors; all 64 lanes active): no old value is kept.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// DPP row broadcast into the rows of ROWMASK; lanes of the other rows receive `id`.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_bcast(double v, double id)
{
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(id), __double2loint(v), CTRL,
                                               ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(id), __double2hiint(v), CTRL,
                                               ROWMASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int OP>
__device__ __forceinline__ constexpr double op_identity()
{
    return OP == OP_SUM ? 0.0 : (OP == OP_MAX ? -__builtin_huge_val() : __builtin_huge_val());
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Reduction within each row of 16 lanes: DPP lane ^ 1 and lane ^ 2 (quad permutes), then
// rotations by 4 and 8; every lane of row r then holds row r's result.
template <int OP>
__device__ __forceinline__ double row_red(double v)
{
    v = comb<OP>(v, dpp_mov<0xB1>(v));    // quad_perm [1,0,3,2]
    v = comb<OP>(v, dpp_mov<0x4E>(v));    // quad_perm [2,3,0,1]
    v = comb<OP>(v, dpp_mov<0x124>(v));   // row_ror:4
    return comb<OP>(v, dpp_mov<0x128>(v));   // row_ror:8
}

// Wave reduction without LDS: row_red, then row r += row r-1 for rows 1 and 3 (broadcast of
// lane 15 of each row) and rows 2, 3 += lane 31; lane 63 then holds
// (row2 + row3) + (row0 + row1).  Every lane returns that value.  Call with all 64 lanes
// active.
template <int OP>
__device__ __forceinline__ double wave_red(double v)
{
    constexpr double id = op_identity<OP>();
    v = row_red<OP>(v);
    v = comb<OP>(v, dpp_bcast<0x142, 0xA>(v, id));   // row_bcast:15 into rows 1, 3
    v = comb<OP>(v, dpp_bcast<0x143, 0xC>(v, id));   // row_bcast:31 into rows 2, 3
    return readlane_d(v, 63);
}

// Inclusive prefix sum over the 64 lanes (lane order): Hillis-Steele shifts by 1, 2, 4, 8
// inside each row of 16 lanes (lanes without a source add 0), then row 1 and row 3 add
// lane 15 of the row below (row broadcast), and rows 2, 3 add lane 31.  Integer, so exact.
__device__ __forceinline__ int wave_scan_incl(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// Reduction of the values of lanes 0..15 (the other lanes' values are ignored): row 0's
// row_red, read from lane 0.  Used where at most 16 values (one per wave) are combined.
template <int OP>
__device__ __forceinline__ double row0_red(double v)
{
    return readlane_d(row_red<OP>(v), 0);
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
    template <int NALL, int I, int OP, int... REST>
    __device__ __forceinline__ static void fold_first(double *v, const double *buf)
    {
        if constexpr (I < NALL) {
            double r = buf[I * NW];
#pragma unroll
            for (int k = 1; k < NW; ++k)
                r = comb<OP>(r, buf[I * NW + k]);
            v[I] = r;
            if constexpr (sizeof...(REST) > 0)
                fold_first<NALL, I + 1, REST...>(v, buf);
        }
    }
    // As run, but only slots 0..NALL-1 are folded in every wave; the other slots are
    // folded in wave 0 only (for thread 0) and are unspecified in the other waves.
    template <int NALL>
    __device__ __forceinline__ static void run_part(double *v, double *lds, int &parity)
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
        if (w == 0)
            fold_all<0, OPS...>(v, buf);
        else if constexpr (NALL > 0)
            fold_first<NALL, 0, OPS...>(v, buf);
    }
    // a single reduction (at a kernel's end) uses only the first buffer: K*NW doubles
    static constexpr int LDS1 = K * NW;
    __device__ __forceinline__ static void run_once(double *v, double *lds)
    {
        int parity = 0;
        run(v, lds, parity);
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

// Stage the high parts (n doubles) and, for tiles with room (LO), the low parts as FP32
// right after them in the dynamic LDS; one barrier.
template <bool LO>
__device__ __forceinline__ void stage_w2(const double *__restrict__ hi,
                                         const double *__restrict__ lo, int n, double *lds)
{
    float *lf = reinterpret_cast<float *>(lds + n);
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        lds[j] = hi[j];
        if constexpr (LO)
            lf[j] = (float)lo[j];
    }
    __syncthreads();
}

// x + wl_j with wl_j from the FP32 copy staged by stage_w2 (after n doubles at `base`)
template <bool LO>
__device__ __forceinline__ double add_lo(double x, const double *base, int n, int j)
{
    if constexpr (LO)
        return x + (double)reinterpret_cast<const float *>(base + n)[j];
    else
        return x;
}

// dynamic LDS of a pass that stages one n-vector of doubles, plus the low parts if LO
__host__ __device__ constexpr size_t lds_w2(int64_t n, bool lo)
{
    return (size_t)n * sizeof(double) + (lo ? (size_t)n * sizeof(float) : 0);
}

// grid(v) = q rint(v / q).  q is a power of two no smaller than the least normal double
// (the API checks this), so 1/q is exact and v (1/q) is v / q rounded once, the same
// value; the compiler hoists 1/q out of the row loops.
__device__ __forceinline__ double grid(double v, double q) { return q * rint(v * (1.0 / q)); }

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

// exp(x) in FP32 for the mixed-precision passes (eval, trial, sparsify).  The FP64
// argument x (as above, <= 709) is split as x/ln2 = kk + f with kk = rint(x/ln2), |f| <= 1/2;
// f is rounded to FP32 (absolute error <= 2^-25), 2^f comes from the hardware base-2
// exponential (v_exp_f32) and 2^kk is applied exactly with ldexp.  The relative error is
// a few FP32 units in the last place whatever |x| is; results below the FP32 range
// (x < about -103) are flushed to 0, and NaN gives 0 as in exp_tab.
constexpr double MX_LOG2E = 0x1.71547652b82fep+0;   // 1 / ln 2
__device__ __forceinline__ float exp_mx(double x)
{
    const double t = fmax(x * MX_LOG2E, -160.0);
    const double kk = rint(t);
    return ldexpf(__builtin_amdgcn_exp2f((float)(t - kk)), (int)kk);
}

// register type of the per-entry values of a pass: FP32 in the mixed-precision form
template <bool MX>
using xval_t = typename std::conditional<MX, float, double>::type;

template <bool MX>
__device__ __forceinline__ double exp_pass(double x, const double *__restrict__ etab)
{
    if constexpr (MX)
        return (double)exp_mx(x);
    else
        return exp_tab(x, etab);
}

// The same values, with the arithmetic skipped where the result is 0 anyway: x <= -746 in
// FP64 (exp underflows past the least subnormal), x <= -110 in the FP32 form; -inf and NaN
// give 0 as before.  A wave whose lanes all fall below skips the exponential (at large
// sigma almost every entry of a row does), so the results are unchanged bit for bit.
template <bool MX>
__device__ __forceinline__ double exp_pass_z(double x, const double *__restrict__ etab)
{
    double r = 0.0;
    if (x > (MX ? -110.0 : -746.0))
        r = exp_pass<MX>(x, etab);
    return r;
}
__device__ __forceinline__ double exp_tab_z(double x, const double *__restrict__ etab)
{
    return exp_pass_z<false>(x, etab);
}

// 2^(j/128), j < 128, into LDS (one barrier)
__device__ __forceinline__ void exp_table_init(double *etab)
{
    for (int j = threadIdx.x; j < EXP_TAB; j += blockDim.x)
        etab[j] = exp2((double)j * (1.0 / EXP_TAB));
    __syncthreads();
}

// log(x) for finite x > 0, table-driven after P. T. P. Tang, "Table-driven implementation
// of the logarithm function in IEEE floating-point arithmetic", ACM TOMS 16(4), 1990, in
// the variant with a tabulated reciprocal: x = 2^e f with f in [1/2, 1); the top six
// fraction bits of f pick interval j, whose centre c_j has the stored reciprocal
// v_j = RN(1/c_j) and the stored L_j = -log(v_j) (computed for the stored v_j, so the
// rounding of 1/c_j costs nothing).  Then f v_j = 1 + r with r = fma(f, v_j, -1),
// |r| <= 2^-7 (+ one rounding, relative 2^-53), and
//   log x = e ln2 + L_j + log1p(r),
// log1p(r) by its Taylor polynomial of degree 8 (remainder below r^9/9 < 2^-66).
// Absolute error about one unit in the last place of max(|log x|, 1/2); subnormal x are
// handled by the hardware frexp.  ltab[2j] = v_j, ltab[2j+1] = L_j, see log_table_init.
constexpr int LOG_TAB = 64;
constexpr double LOG_LN2_HI = 0x1.62e42fefa39efp-1;    // ln 2, rounded
constexpr double LOG_LN2_LO = 0x1.abc9e3b39803fp-56;   // ln 2 - LOG_LN2_HI

__device__ __forceinline__ double log_tab(double x, const double *__restrict__ ltab)
{
    const double f = __builtin_amdgcn_frexp_mant(x);   // [1/2, 1)
    const int e = __builtin_amdgcn_frexp_exp(x);
    const int j = (__double2hiint(f) >> 14) & (LOG_TAB - 1);
    const double2 t = reinterpret_cast<const double2 *>(ltab)[j];
    const double r = fma(f, t.x, -1.0);
    double q = fma(r, -1.0 / 8.0, 1.0 / 7.0);
    q = fma(q, r, -1.0 / 6.0);
    q = fma(q, r, 1.0 / 5.0);
    q = fma(q, r, -1.0 / 4.0);
    q = fma(q, r, 1.0 / 3.0);
    q = fma(q, r, -0.5);
    const double p = fma(r * r, q, r);                   // log1p(r)
    const double ed = (double)e;
    return fma(ed, LOG_LN2_HI, t.y) + fma(ed, LOG_LN2_LO, p);
}

// (v_j, L_j) for j < 64 into LDS (2 * LOG_TAB doubles, 16-byte aligned); the caller's
// next barrier publishes it.  c_j = (1 + (j + 1/2)/64) / 2 is the centre of the j-th of the
// 64 equal parts of [1/2, 1).
__device__ __forceinline__ void log_table_init(double *ltab)
{
    for (int j = threadIdx.x; j < LOG_TAB; j += blockDim.x) {
        const double c = 0.5 * (1.0 + ((double)j + 0.5) * (1.0 / LOG_TAB));
        const double v = 1.0 / c;
        ltab[2 * j] = v;
        ltab[2 * j + 1] = -log(v);
    }
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
template <int NT, int Q, int QF, int VEC, bool VECOK, bool PREFETCH, int RC, typename CT,
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
            const int slot = (i - i0) & (RC - 1);
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
            const int slot = (i - i0) & (RC - 1);
            if (slot == 0)
                stage(i);
            load_row<NT, Q, QF, VEC, VECOK>(C + (int64_t)i * ldc, n, xr);
            body(i, slot, xr);
        }
    }
}

// Cost formed from points (no stored matrix): the kernels' cost type is the tag PtsCost<DIM>,
// their C argument points to x (m x DIM) and py / pscale give y (n x DIM) and the scale.
// C_ij = pscale * ((x_i1 - y_j1)^2 + (x_i2 - y_j2)^2 [+ (x_i3 - y_j3)^2]), every product
// and sum rounded separately in that order.
template <int DIM>
struct PtsCost {};
template <typename CT>
struct IsPts : std::false_type {};
template <int DIM>
struct IsPts<PtsCost<DIM>> : std::true_type {
    static constexpr int dim = DIM;
};

template <int DIM>
__device__ __forceinline__ double pts_cost(const double *xi, const double *yj, double scale)
{
#pragma clang fp contract(off)
    const double t0 = xi[0] - yj[0];
    double s = t0 * t0;
    const double t1 = xi[1] - yj[1];
    s = s + t1 * t1;
    if constexpr (DIM == 3) {
        const double t2 = xi[2] - yj[2];
        s = s + t2 * t2;
    }
    return s * scale;
}

// Row loop over a points cost: each thread keeps y of its own columns in registers (slots
// past n use column n - 1, as load_row does) and forms every row from x_i, so the pass
// reads no m x n array.
template <int NT, int Q, int QF, int DIM, int RC, typename Stage, typename Body>
__device__ __forceinline__ void row_loop_pts(const double *__restrict__ x,
                                             const double *__restrict__ y, double scale, int n,
                                             int i0, int i1, Stage &stage, Body &body)
{
    constexpr int E = Q * 2;
    double yr[E * DIM];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = min(col_of<NT, 2>(e), n - 1);
#pragma unroll
        for (int k = 0; k < DIM; ++k)
            yr[e * DIM + k] = y[(int64_t)j * DIM + k];
    }
    double xr[E];
    for (int i = i0; i < i1; ++i) {
        const int slot = (i - i0) & (RC - 1);
        if (slot == 0)
            stage(i);
        double xi[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k)
            xi[k] = x[(int64_t)i * DIM + k];
#pragma unroll
        for (int e = 0; e < E; ++e)
            xr[e] = pts_cost<DIM>(xi, yr + e * DIM, scale);
        body(i, slot, xr);
    }
}

// 16-byte vector loads when the matrix start and the row pitch are 16-byte aligned and n
// is a multiple of VEC (the same for every row); scalar loads otherwise.
// PREFETCH = false (passes whose per-entry state leaves no registers for a second row):
// each row is loaded when it is reached.
// RC: rows per staged chunk (a power of two; the kernel's stage_rows<RC> fills them).
template <int NT, int Q, int QF, int VEC, bool PREFETCH = true, int RC = ROWCH, typename CT,
          typename Stage, typename Body>
__device__ __forceinline__ void row_loop(const CT *__restrict__ C, int64_t ldc,
                                         const double *__restrict__ py, double pscale, int n,
                                         int i0, int i1, Stage &&stage, Body &&body)
{
    if constexpr (IsPts<CT>::value) {
        row_loop_pts<NT, Q, QF, IsPts<CT>::dim, RC>(reinterpret_cast<const double *>(C), py,
                                                    pscale, n, i0, i1, stage, body);
        return;
    } else {
    const bool vec_ok = (reinterpret_cast<uintptr_t>(C) & 15u) == 0 &&
                        ((uint64_t)ldc * sizeof(CT)) % 16 == 0 && n % VEC == 0;
    if (vec_ok)
        row_loop_v<NT, Q, QF, VEC, true, PREFETCH, RC>(C, ldc, n, i0, i1, stage, body);
    else
        row_loop_v<NT, Q, QF, VEC, false, PREFETCH, RC>(C, ldc, n, i0, i1, stage, body);
    }
}

// Copy rows [i, min(i + RC, i1)) of up to four m-vectors into LDS (null: skipped).
template <int RC = ROWCH>
__device__ __forceinline__ void stage_rows(int i, int i1, const double *__restrict__ s0,
                                           double *d0, const double *__restrict__ s1, double *d1,
                                           const double *__restrict__ s2, double *d2,
                                           const double *__restrict__ s3 = nullptr,
                                           double *d3 = nullptr)
{
    __syncthreads();   // the previous chunk may still be read
    const int cnt = min(RC, i1 - i);
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

// Host side: a launch of `fn` with `dyn` bytes of dynamic LDS fits the device's LDS per
// workgroup (its static LDS included).  hipErrorInvalidConfiguration otherwise, so that an
// oversized request fails as an error instead of reaching the hardware.  `cache` (one per
// launch site) keeps the kernel's static LDS size after the first query.
struct LdsCache {
    std::atomic<long> static_bytes{-1};
};
inline hipError_t lds_check(const void *fn, size_t dyn, LdsCache &cache)
{
    static std::atomic<int> max_lds[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= 64)
        return hipErrorInvalidDevice;
    int lim = max_lds[dev].load(std::memory_order_relaxed);
    if (lim <= 0) {
        e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess)
            return e;
        max_lds[dev].store(lim, std::memory_order_relaxed);
    }
    long st = cache.static_bytes.load(std::memory_order_relaxed);
    if (st < 0) {
        hipFuncAttributes fa;
        e = hipFuncGetAttributes(&fa, fn);
        if (e != hipSuccess)
            return e;
        st = (long)fa.sharedSizeBytes;
        cache.static_bytes.store(st, std::memory_order_relaxed);
    }
    return (size_t)st + dyn <= (size_t)lim ? hipSuccess : hipErrorInvalidConfiguration;
}

}  // namespace

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

// the same with the precision form as a second compile-time choice (constexpr bool MX)
#define IBSN_DISPATCH_MX(NT_, Q_, QF_, BODY)                                      \
    if (p.nt == NT_ && p.q == Q_ && p.qf == QF_) {                               \
        constexpr int NT = NT_, Q = Q_, QF = QF_;                                \
        if (d.cost_kind == 0) {                                                  \
            constexpr int VEC = 2;                                               \
            using CT = double;                                                   \
            if (d.mixed) {                                                       \
                constexpr bool MX = true;                                        \
                BODY;                                                            \
            } else {                                                             \
                constexpr bool MX = false;                                       \
                BODY;                                                            \
            }                                                                    \
        } else if (d.cost_kind == 1) {                                           \
            constexpr int VEC = 4;                                               \
            using CT = float;                                                    \
            if (d.mixed) {                                                       \
                constexpr bool MX = true;                                        \
                BODY;                                                            \
            } else {                                                             \
                constexpr bool MX = false;                                       \
                BODY;                                                            \
            }                                                                    \
        } else if (d.pdim == 2) {                                                \
            constexpr int VEC = 2;                                               \
            using CT = PtsCost<2>;                                               \
            if (d.mixed) {                                                       \
                constexpr bool MX = true;                                        \
                BODY;                                                            \
            } else {                                                             \
                constexpr bool MX = false;                                       \
                BODY;                                                            \
            }                                                                    \
        } else {                                                                 \
            constexpr int VEC = 2;                                               \
            using CT = PtsCost<3>;                                               \
            if (d.mixed) {                                                       \
                constexpr bool MX = true;                                        \
                BODY;                                                            \
            } else {                                                             \
                constexpr bool MX = false;                                       \
                BODY;                                                            \
            }                                                                    \
        }                                                                        \
        return hipGetLastError();                                                \
    }

#define IBSN_DISPATCH(NT_, Q_, QF_, BODY)                                         \
    if (p.nt == NT_ && p.q == Q_ && p.qf == QF_) {                               \
        constexpr int NT = NT_, Q = Q_, QF = QF_;                                \
        if (d.cost_kind == 0) {                                                  \
            constexpr int VEC = 2;                                               \
            using CT = double;                                                   \
            BODY;                                                                \
        } else if (d.cost_kind == 1) {                                           \
            constexpr int VEC = 4;                                               \
            using CT = float;                                                    \
            BODY;                                                                \
        } else if (d.pdim == 2) {                                                \
            constexpr int VEC = 2;                                               \
            using CT = PtsCost<2>;                                               \
            BODY;                                                                \
        } else {                                                                 \
            constexpr int VEC = 2;                                               \
            using CT = PtsCost<3>;                                               \
            BODY;                                                                \
        }                                                                        \
        return hipGetLastError();                                                \
    }

}  // namespace ibsn
