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

template <int OP>
__device__ __forceinline__ double wave_red(double v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1)
        v = comb<OP>(v, __shfl_xor(v, o, WAVE));
    return v;
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

// Load row `row` (n entries) into x[Q*VEC] (cost type); entries past n read as 0.
// A row that starts on a 16-byte boundary is read with 16-byte vector loads; any other
// row (odd leading dimension) with scalar loads of the same columns.
template <int NT, int Q, int VEC, typename CT>
__device__ __forceinline__ void load_row(const CT *__restrict__ row, int n, CT *x)
{
    if ((reinterpret_cast<uintptr_t>(row) & 15u) == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int j0 = (q * NT + (int)threadIdx.x) * VEC;
            if (j0 + VEC <= n) {
                VecLoad<CT, VEC>::get(row + j0, x + q * VEC);
            } else {
#pragma unroll
                for (int v = 0; v < VEC; ++v)
                    x[q * VEC + v] = (j0 + v < n) ? row[j0 + v] : CT(0);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int j0 = (q * NT + (int)threadIdx.x) * VEC;
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                x[q * VEC + v] = (j0 + v < n) ? row[j0 + v] : CT(0);
        }
    }
}

template <int NT, int Q, int VEC>
__device__ __forceinline__ void load_cols(const double *__restrict__ src, int n, double *x)
{
#pragma unroll
    for (int e = 0; e < Q * VEC; ++e) {
        const int j = col_of<NT, VEC>(e);
        x[e] = j < n ? src[j] : 0.0;
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

__device__ __forceinline__ void row_range(int m, int &i0, int &i1)
{
    const int64_t g = blockIdx.x, G = gridDim.x;
    i0 = (int)((int64_t)m * g / G);
    i1 = (int)((int64_t)m * (g + 1) / G);
}

// ---------------------------------------------------------------------------------
// eval: M_i = max_j theta_ij, S_i = sum_j exp(theta_ij - M_i), column partials of
// a_i P_ij, objective row terms a_i ((r_i + M_i) + log S_i).
// ---------------------------------------------------------------------------------
template <int NT, int Q, int VEC, typename CT>
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
    using RedMax = BlockRed<NT, OP_MAX>;
    using RedSum = BlockRed<NT, OP_SUM>;
    __shared__ double lds[RedMax::LDS];
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    double wr[E], acc[E], x[E];
    CT xr[E], xn[E];
    load_cols<NT, Q, VEC>(w, n, wr);
#pragma unroll
    for (int e = 0; e < E; ++e)
        acc[e] = 0.0;
    double rowacc = 0.0;
    if (i0 < i1)
        load_row<NT, Q, VEC>(C + (int64_t)i0 * ldc, n, xr);
    for (int i = i0; i < i1; ++i) {
        if (i + 1 < i1)
            load_row<NT, Q, VEC>(C + (int64_t)(i + 1) * ldc, n, xn);
        double red[1] = {-INFINITY};
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double th =
                col_of<NT, VEC>(e) < n ? fma(-sigma, (double)xr[e], wr[e]) : -INFINITY;
            red[0] = fmax(red[0], th);
        }
        RedMax::run(red, lds, parity);
        const double M = grid(red[0], qg);
        red[0] = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double p =
                col_of<NT, VEC>(e) < n ? exp(fma(-sigma, (double)xr[e], wr[e] - M)) : 0.0;
            x[e] = p;
            red[0] += p;
        }
        RedSum::run(red, lds, parity);
        const double S = red[0];
        const double ai = a[i];
        const double sc = ai / S;
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
                rowacc += ai * ((r[i] + M) + ls);
        }
#pragma unroll
        for (int e = 0; e < E; ++e)
            xr[e] = xn[e];
    }
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
template <int NT, int Q, int VEC, typename CT, int BIG>
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
    double wr[E], acc[E], x[E];
    CT xr[E], xn[E];
    load_cols<NT, Q, VEC>(w, n, wr);
    stage_lds(colv, n, cvl);
#pragma unroll
    for (int e = 0; e < E; ++e)
        acc[e] = 0.0;
    double rowacc = 0.0;
    if (i0 < i1)
        load_row<NT, Q, VEC>(C + (int64_t)i0 * ldc, n, xr);
    for (int i = i0; i < i1; ++i) {
        if (i + 1 < i1)
            load_row<NT, Q, VEC>(C + (int64_t)(i + 1) * ldc, n, xn);
        const double Mi = Mb[i];
        double red[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = col_of<NT, VEC>(e);
            if (j < n) {
                const double q = exp(fma(-sigma, (double)xr[e], wr[e] - Mi));
                const double cv = cvl[j];
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
            } else {
                x[e] = 0.0;
            }
        }
        Red::run(red, lds, parity);
        const double A = red[0], B = red[1], Z = red[2], mx = red[3];
        const double ai = a[i];
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
#pragma unroll
        for (int e = 0; e < E; ++e)
            xr[e] = xn[e];
    }
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
template <int NT, int Q, int VEC, typename CT>
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
    double acc[E], x[E];
    CT xr[E], xn[E];
    const int istar = *istar_p;
    stage_lds(w, n, wl);
#pragma unroll
    for (int e = 0; e < E; ++e)
        acc[e] = 0.0;
    if (i0 < i1)
        load_row<NT, Q, VEC>(C + (int64_t)i0 * ldc, n, xr);
    for (int i = i0; i < i1; ++i) {
        if (i + 1 < i1)
            load_row<NT, Q, VEC>(C + (int64_t)(i + 1) * ldc, n, xn);
        const double Mi = M[i], Si = S[i];
        const bool dense = (i == istar);
        int *cn = cnt[i & 1];
        double red[1] = {0.0};
        unsigned long long keepbits = 0;
        unsigned long long bal[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = col_of<NT, VEC>(e);
            const bool valid = j < n;
            const double p = valid ? exp(fma(-sigma, (double)xr[e], wl[j] - Mi)) / Si : 0.0;
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
        const double kappa = red[0];
        int running = 0, base[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            for (int k = 0; k < NW; ++k) {
                if (k == wv)
                    base[q] = running;
                running += cn[q * NW + k];
            }
        }
        const double ai = a[i];
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
                    const double pv = dense ? x[e] : x[e] / kappa;
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
#pragma unroll
        for (int e = 0; e < E; ++e)
            xr[e] = xn[e];
    }
    store_cols<NT, Q, VEC>(colpart + (int64_t)blockIdx.x * n, n, acc);
}

// ---------------------------------------------------------------------------------
// Stop test pass 1 (Algorithm 3, steps 2-8): X = a_i P; z_i; column sums of X and z X.
// ---------------------------------------------------------------------------------
template <int NT, int Q, int VEC, typename CT>
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
    int parity = 0;
    int i0, i1;
    row_range(m, i0, i1);
    extern __shared__ double wl[];   // w staged in LDS (n doubles)
    double ax[E], az[E], x[E];
    CT xr[E], xn[E];
    stage_lds(w, n, wl);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        ax[e] = 0.0;
        az[e] = 0.0;
    }
    double rowacc = 0.0;
    if (i0 < i1)
        load_row<NT, Q, VEC>(C + (int64_t)i0 * ldc, n, xr);
    for (int i = i0; i < i1; ++i) {
        if (i + 1 < i1)
            load_row<NT, Q, VEC>(C + (int64_t)(i + 1) * ldc, n, xn);
        const double Mi = M[i], Si = S[i], ai = a[i];
        double red[1] = {0.0};
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = col_of<NT, VEC>(e);
            const double X =
                j < n ? ai * (exp(fma(-sigma, (double)xr[e], wl[j] - Mi)) / Si) : 0.0;
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
#pragma unroll
        for (int e = 0; e < E; ++e)
            xr[e] = xn[e];
    }
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
template <int NT, int Q, int VEC, typename CT>
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
    stage_lds(w, n, wl);
    double X[E];
    CT cst[E];
    double t_dphi = 0.0, t_cxh = 0.0, t_cx = 0.0, t_xu = 0.0, t_xhmin = INFINITY, t_xf = 0.0,
           t_cf = 0.0;
    double azg = 0.0, azp = 0.0;
    for (int i = i0; i < i1; ++i) {
        load_row<NT, Q, VEC>(C + (int64_t)i * ldc, n, cst);
        const double Mi = M[i], Si = S[i], ai = a[i], zi = z[i];
        double red[3] = {0.0, INFINITY, INFINITY};
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = col_of<NT, VEC>(e);
            if (j < n) {
                const double c = (double)cst[e];
                const double Xv = ai * (exp(fma(-sigma, c, wl[j] - Mi)) / Si);
                X[e] = Xv;
                red[0] = fma(Xv, y[j], red[0]);
                red[1] = fmin(red[1], c - gamma[j]);
                red[2] = fmin(red[2], c - psi[j]);
            } else {
                X[e] = 0.0;
            }
        }
        Red3::run(red, lds, parity);
        const double eri = fmax(ai - zi * red[0], 0.0);   // >= 0 exactly; clamp rounding
        const double zg = red[1], zp = red[2];
        const double la = log(ai), ls = log(Si);
#pragma unroll 2
        for (int e = 0; e < E; ++e) {
            const int j = col_of<NT, VEC>(e);
            if (j < n) {
                const double c = (double)cst[e];
                const double Xv = X[e];
                const double f = (zi * Xv) * y[j];
                const double xh = er1 > 0.0 ? f + eri * ec[j] / er1 : f;
                if (xh > 0.0) {
                    const double lx = la + fma(-sigma, c, wl[j] - Mi) - ls;
                    t_dphi += xh * (log(xh) - lx) - xh + Xv;
                } else {
                    t_dphi += Xv;
                }
                t_cxh = fma(c, xh, t_cxh);
                t_cx = fma(c, Xv, t_cx);
                t_xhmin = fmin(t_xhmin, xh);
                t_xu = fma(Xv, (c - gamma[j]) - zg, t_xu);
                t_xf = fma(Xv, Xv, t_xf);
                t_cf = fma(c, c, t_cf);
                if (xhat)
                    xhat[(int64_t)i * n + j] = xh;
            }
        }
        if (threadIdx.x == 0) {
            azg += ai * zg;
            azp += ai * zp;
        }
    }
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
#define IBSN_ROW_CONFIGS(X) \
    X(256, 1)               \
    X(256, 2)               \
    X(256, 4)               \
    X(512, 4)               \
    X(512, 6)               \
    X(512, 8)               \
    X(512, 10)

bool plan_rows(int64_t m, int64_t n, int cost_kind, int num_cus, RowPlan *p)
{
    static const int cfg[][2] = {{256, 1}, {256, 2}, {256, 4}, {512, 4},
                                 {512, 6}, {512, 8}, {512, 10}};
    const int vec = cost_kind == 1 ? 4 : 2;
    for (const auto &c : cfg) {
        if ((int64_t)c[0] * c[1] * vec >= n) {
            p->nt = c[0];
            p->q = c[1];
            p->vec = vec;
            const int per_cu = c[0] == 512 ? 1 : 4;
            int64_t g = (int64_t)num_cus * per_cu;
            p->grid = (int)(g < m ? g : m);
            return true;
        }
    }
    return false;
}

#define IBSN_DISPATCH(NT_, Q_, BODY64, BODY32)          \
    if (p.nt == NT_ && p.q == Q_) {                    \
        if (d.cost_kind == 0) {                        \
            constexpr int NT = NT_, Q = Q_, VEC = 2;   \
            using CT = double;                         \
            BODY64;                                    \
        } else {                                       \
            constexpr int NT = NT_, Q = Q_, VEC = 4;   \
            using CT = float;                          \
            BODY32;                                    \
        }                                              \
        return hipGetLastError();                      \
    }

hipError_t launch_eval(const RowPlan &p, const DenseArgs &d, const double *r, double *M, double *S,
                       double *lse, double *plan, double *colpart, double *rowpart, hipStream_t st)
{
#define BODY                                                                                     \
    hipLaunchKernelGGL((k_eval<NT, Q, VEC, CT>), dim3(p.grid), dim3(NT), 0, st,                  \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.q, d.w, d.a, r, M, S, \
                       lse,                                                                      \
                       plan, colpart, rowpart)
#define X(a, b) IBSN_DISPATCH(a, b, BODY, BODY)
    IBSN_ROW_CONFIGS(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

hipError_t launch_trial(const RowPlan &p, const DenseArgs &d, const double *M, const double *colv,
                        const double *scal, double *M_new, double *S_new, double *colpart,
                        double *rowpart, hipStream_t st)
{
    const size_t lds_bytes = (size_t)d.n * sizeof(double);
#define BODY                                                                                      \
    hipLaunchKernelGGL((k_trial<NT, Q, VEC, CT, 0>), dim3(p.grid), dim3(NT), lds_bytes, st,       \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.q, d.w, d.a, M, colv, \
                       scal, M_new, S_new, colpart, rowpart);                                     \
    hipLaunchKernelGGL((k_trial<NT, Q, VEC, CT, 1>), dim3(p.grid), dim3(NT), lds_bytes, st,       \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.q, d.w, d.a, M, colv, \
                       scal, M_new, S_new, colpart, rowpart)
#define X(a, b) IBSN_DISPATCH(a, b, BODY, BODY)
    IBSN_ROW_CONFIGS(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

hipError_t launch_sparsify(const RowPlan &p, const DenseArgs &d, const double *M, const double *S,
                           double rho, const int *istar, int32_t *col, double *val, int32_t *len,
                           double *colpart, hipStream_t st)
{
    const size_t lds_bytes = (size_t)d.n * sizeof(double);
#define BODY                                                                                     \
    hipLaunchKernelGGL((k_sparsify<NT, Q, VEC, CT>), dim3(p.grid), dim3(NT), lds_bytes, st,              \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.w, d.a, M, S, rho, \
                       istar, col, val, len, colpart)
#define X(a, b) IBSN_DISPATCH(a, b, BODY, BODY)
    IBSN_ROW_CONFIGS(X)
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
    hipLaunchKernelGGL((k_stop1<NT, Q, VEC, CT>), dim3(p.grid), dim3(NT), lds_bytes, st,                 \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.w, d.a, M, S, z,   \
                       colpart, colpart2, rowpart)
#define X(a, b) IBSN_DISPATCH(a, b, BODY, BODY)
    IBSN_ROW_CONFIGS(X)
#undef X
#undef BODY
    return hipErrorInvalidValue;
}

hipError_t launch_stop2(const RowPlan &p, const DenseArgs &d, const double *M, const double *S,
                        const Stop2Vec &v, double *xhat, double *rowpart, hipStream_t st)
{
    const size_t lds_bytes = (size_t)d.n * sizeof(double);
#define BODY                                                                                      \
    hipLaunchKernelGGL((k_stop2<NT, Q, VEC, CT>), dim3(p.grid), dim3(NT), lds_bytes, st,                  \
                       (const CT *)d.C, d.ldc, (int)d.m, (int)d.n, d.sigma, d.w, d.a, M, S,       \
                       v.gamma, v.psi, v.y, v.ec, v.z, v.er1, xhat, rowpart)
#define X(a, b) IBSN_DISPATCH(a, b, BODY, BODY)
    IBSN_ROW_CONFIGS(X)
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
