// solver_kernels.hip -- n- and m-vector steps of the IBSN iteration (Algorithm 2) that
// sit between the dense passes: norms of g, the Sinkhorn gamma-step with centring,
// the Armijo column factors, the rounding vectors of Algorithm 3, the certificate
// finalisation and the outer update of the implicit prox centre.
//
// Each reduction runs in one workgroup of 1024 threads with a fixed summation order
// (thread-strided partial sums, then a butterfly and an ordered fold), so results do
// not depend on timing.  Scalars are exchanged through a small device array `scal`.
#include "ibsn_internal.h"
#include "solver_kernels.h"

#include <math.h>

namespace ibsn {
namespace {

constexpr int WAVE = 64;
constexpr int NT = 1024;
constexpr int NW = NT / WAVE;

template <int OP>
__device__ __forceinline__ double comb(double x, double y)
{
    if constexpr (OP == 0)
        return x + y;
    else if constexpr (OP == 1)
        return fmax(x, y);
    else
        return fmin(x, y);
}

// reduction over the 1024 threads; result in every thread
template <int OP>
__device__ __forceinline__ double wg_red(double v, double *lds)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1)
        v = comb<OP>(v, __shfl_xor(v, o, WAVE));
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0)
        lds[threadIdx.x / WAVE] = v;
    __syncthreads();
    double r = lds[0];
#pragma unroll
    for (int k = 1; k < NW; ++k)
        r = comb<OP>(r, lds[k]);
    return r;
}

// scal[SC_GN2] = ||g||^2, scal[SC_G1] = ||g||_1, scal[SC_GN] = ||g||
__global__ __launch_bounds__(NT) void k_gnorms(int n, const double *__restrict__ g,
                                               double *__restrict__ scal)
{
    __shared__ double lds[NW];
    double s2 = 0.0, s1 = 0.0;
    for (int j = threadIdx.x; j < n; j += NT) {
        const double v = g[j];
        s2 = fma(v, v, s2);
        s1 += fabs(v);
    }
    s2 = wg_red<0>(s2, lds);
    s1 = wg_red<0>(s1, lds);
    if (threadIdx.x == 0) {
        scal[SC_GN2] = s2;
        scal[SC_GN] = sqrt(s2);
        scal[SC_G1] = s1;
    }
}

__device__ __forceinline__ double grid(double v, double q) { return q * rint(v / q); }

// Add d to the two-level potential (wh, wl): u = wl + d with its rounding error e (two-sum),
// wh += grid(u) (exact: both on the grid), wl = (u - grid(u)) + e.  With wl = 0 and d on the
// grid (potentials kept on the grid) this is wh += d, wl = 0.
__device__ __forceinline__ void dd_add(double &wh, double &wl, double d, double q)
{
    const double u = wl + d;
    const double bb = u - wl;
    const double e = (wl - (u - bb)) + (d - bb);
    const double g = grid(u, q);
    wh += g;
    wl = (u - g) + e;
}

// Sinkhorn gamma-step on Z^k with zeta = zeta(gamma) (eq. (4), (5)):
// gamma_j += eta (log b_j - log c_j), taken on the potentials w = s + gamma/eta as
// w_j += log b_j - lc_j with lc_j = log c_j (split = 0: the step rounded to the grid); then
// gamma = eta (w - s) is centred (Algorithm 2, step 4) by a common shift of w, which leaves
// P unchanged.
__global__ __launch_bounds__(NT) void k_sinkhorn_step(int n, double eta, double q, int split,
                                                      const double *__restrict__ b,
                                                      const double *__restrict__ lc,
                                                      const double *__restrict__ s,
                                                      double *__restrict__ w,
                                                      double *__restrict__ wlo)
{
    __shared__ double lds[NW];
    double acc = 0.0;
    for (int j = threadIdx.x; j < n; j += NT) {
        const double d0 = log(b[j]) - lc[j];
        double wh = w[j], wl = wlo[j];
        dd_add(wh, wl, split ? d0 : grid(d0, q), q);
        w[j] = wh;
        wlo[j] = wl;
        acc += eta * ((wh - s[j]) + wl);
    }
    acc = wg_red<0>(acc, lds);
    const double sh0 = (acc / (double)n) / eta;
    const double sh = split ? -sh0 : -grid(sh0, q);
    for (int j = threadIdx.x; j < n; j += NT) {
        double wh = w[j], wl = wlo[j];
        dd_add(wh, wl, sh, q);
        w[j] = wh;
        wlo[j] = wl;
    }
}

// (wh, wl) += d over n columns (the accepted Newton step)
__global__ __launch_bounds__(256) void k_dd_axpy(int n, double q, const double *__restrict__ d,
                                                 double *__restrict__ w, double *__restrict__ wlo)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) {
        double wh = w[j], wl = wlo[j];
        dd_add(wh, wl, d[j], q);
        w[j] = wh;
        wlo[j] = wl;
    }
}

// log c_j from the eval's column sums (the Sinkhorn step's lc)
__global__ __launch_bounds__(256) void k_log(int n, const double *__restrict__ c,
                                             double *__restrict__ lc)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n)
        lc[j] = log(c[j]);
}

// scal[SC_WMAX] = max_j |s_j + gamma_j / eta|
__global__ __launch_bounds__(NT) void k_wmax(int n, const double *__restrict__ s,
                                             const double *__restrict__ gamma, double eta,
                                             double *__restrict__ scal)
{
    __shared__ double lds[NW];
    double mx = 0.0;
    for (int j = threadIdx.x; j < n; j += NT)
        mx = fmax(mx, fabs(s[j] + gamma[j] / eta));
    mx = wg_red<1>(mx, lds);
    if (threadIdx.x == 0)
        scal[SC_WMAX] = mx;
}

// per-workgroup max |C| over a block of rows -> part[g]
__device__ __forceinline__ double cost_from_points(const double *__restrict__ x,
                                                   const double *__restrict__ y, int dim,
                                                   double scale, int64_t i, int64_t j)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int k = 0; k < dim; ++k) {
        const double t = x[i * dim + k] - y[j * dim + k];
        s = k == 0 ? t * t : s + t * t;
    }
    return s * scale;
}

// kind 2 (points): C is x (m x ldc), y and scale give the cost
__global__ __launch_bounds__(256) void k_cost_max_part(int m, int n, int64_t ldc, int kind,
                                                       const void *__restrict__ C,
                                                       const double *__restrict__ py,
                                                       double pscale,
                                                       double *__restrict__ part)
{
    __shared__ double lds[4];
    const int64_t g = blockIdx.x, G = gridDim.x;
    const int i0 = (int)((int64_t)m * g / G), i1 = (int)((int64_t)m * (g + 1) / G);
    double mx = 0.0;
    for (int i = i0; i < i1; ++i)
        for (int j = threadIdx.x; j < n; j += 256) {
            const double c =
                kind == 2   ? cost_from_points((const double *)C, py, (int)ldc, pscale, i, j)
                : kind == 1 ? (double)((const float *)C)[(int64_t)i * ldc + j]
                            : ((const double *)C)[(int64_t)i * ldc + j];
            // a NaN or infinite entry makes the maximum +inf (fmax would drop a NaN)
            mx = fabs(c) <= 1.7976931348623157e308 ? fmax(mx, fabs(c)) : INFINITY;
        }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1)
        mx = fmax(mx, __shfl_xor(mx, o, WAVE));
    if ((threadIdx.x & (WAVE - 1)) == 0)
        lds[threadIdx.x / WAVE] = mx;
    __syncthreads();
    if (threadIdx.x == 0)
        part[g] = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
}

// gamma = eta (w - s) with w = wh + wl (wh - s is exact: both are grid values of the
// outer iteration or earlier ones, and their difference is small)
__global__ __launch_bounds__(256) void k_gamma_of(int n, double eta, const double *__restrict__ w,
                                                  const double *__restrict__ wlo,
                                                  const double *__restrict__ s,
                                                  double *__restrict__ gamma)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n)
        gamma[j] = eta * ((w[j] - s[j]) + wlo[j]);
}

__global__ __launch_bounds__(NT) void k_center(int n, double *__restrict__ gamma)
{
    __shared__ double lds[NW];
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += NT)
        s += gamma[j];
    s = wg_red<0>(s, lds);
    const double mean = s / (double)n;
    for (int j = threadIdx.x; j < n; j += NT)
        gamma[j] -= mean;
}

// Armijo step tau_j = t Delta_j / eta (split = 0: rounded to the grid, tau_j =
// grid(t Delta_j / eta)); the trial point is w + tau, which the accepted step forms exactly
// as a two-level potential.  Column factors: small step (max tau <= 500): colv = expm1(tau), shift 0;
// big step: colv = exp(tau - max tau), shift = max tau.  scal[SC_TB] = b^T tau.
// scal[SC_BIG] = 0 (max tau <= 80), 2 (80 < max tau <= 500: small form, but q e^tau can
// exceed FLT_MAX, so the mixed form hands such a step to the FP64 pass) or 1 (big step).
__global__ __launch_bounds__(NT) void k_trial_prep(int n, double t, double eta, double q, int split,
                                                   const double *__restrict__ Delta,
                                                   const double *__restrict__ b,
                                                   double *__restrict__ tau,
                                                   double *__restrict__ colv,
                                                   double *__restrict__ scal)
{
    __shared__ double lds[NW];
    double mx = -INFINITY, bt = 0.0;
#pragma unroll 4   // one workgroup: keep several loads in flight per thread
    for (int j = threadIdx.x; j < n; j += NT) {
        const double v0 = t * Delta[j] / eta;
        const double v = split ? v0 : grid(v0, q);
        tau[j] = v;
        mx = fmax(mx, v);
        bt = fma(b[j], v, bt);
    }
    mx = wg_red<1>(mx, lds);
    bt = wg_red<0>(bt, lds);
    const bool big = mx > 500.0;
#pragma unroll 4
    for (int j = threadIdx.x; j < n; j += NT) {
        const double v = tau[j];
        colv[j] = big ? exp(v - mx) : expm1(v);
    }
    if (threadIdx.x == 0) {
        scal[SC_BIG] = big ? 1.0 : (mx > 80.0 ? 2.0 : 0.0);
        scal[SC_TAUSHIFT] = big ? mx : 0.0;
        scal[SC_TB] = bt;
    }
}

// sum of G per-workgroup values (fixed order) combined into an objective-type scalar:
// scal[slot] = alpha * sum_g part[g*stride + off] + beta * scal[src]
__global__ __launch_bounds__(NT) void k_sum_parts(int G, int stride, int off,
                                                  const double *__restrict__ part, double alpha,
                                                  double beta, int src, int slot, int op,
                                                  double *__restrict__ scal)
{
    __shared__ double lds[NW];
    double s = op == 0 ? 0.0 : (op == 1 ? -INFINITY : INFINITY);
    for (int g = threadIdx.x; g < G; g += NT) {
        const double v = part[(int64_t)g * stride + off];
        s = op == 0 ? s + v : (op == 1 ? fmax(s, v) : fmin(s, v));
    }
    if (op == 0)
        s = wg_red<0>(s, lds);
    else if (op == 1)
        s = wg_red<1>(s, lds);
    else
        s = wg_red<2>(s, lds);
    if (threadIdx.x == 0)
        scal[slot] = alpha * s + (src >= 0 ? beta * scal[src] : 0.0);
}

// dot product into scal[slot]: x.y (or sum x if y == null)
__global__ __launch_bounds__(NT) void k_dot_slot(int n, const double *__restrict__ x,
                                                 const double *__restrict__ y, int slot,
                                                 double *__restrict__ scal)
{
    __shared__ double lds[NW];
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += NT)
        s = y ? fma(x[j], y[j], s) : s + x[j];
    s = wg_red<0>(s, lds);
    if (threadIdx.x == 0)
        scal[slot] = s;
}

__global__ void k_fill(int n, double v, double *__restrict__ x)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n)
        x[j] = v;
}

// Algorithm 3 vectors after pass 1: y_j = min(b_j / colX_j, 1), e_c = b - y.colF,
// ||e_r||_1 = sum a - sum_j y_j colF_j (sum of the rows of F), psi_j = (w_j - log b_j)/sigma
// with w = wh + wl, column residual sum_j (colX_j - b_j)^2, b^T gamma, b^T psi.
__global__ __launch_bounds__(NT) void k_stop_prep(int n, double sigma, const double *__restrict__ b,
                                                  const double *__restrict__ w,
                                                  const double *__restrict__ wlo,
                                                  const double *__restrict__ gamma,
                                                  const double *__restrict__ colX,
                                                  const double *__restrict__ colF,
                                                  double *__restrict__ y, double *__restrict__ ec,
                                                  double *__restrict__ psi,
                                                  double *__restrict__ scal)
{
    __shared__ double lds[NW];
    double syf = 0.0, cc = 0.0, bg = 0.0, bp = 0.0;
#pragma unroll 4   // one workgroup: keep several loads in flight per thread
    for (int j = threadIdx.x; j < n; j += NT) {
        const double bj = b[j], cx = colX[j], cf = colF[j];
        const double yj = fmin(bj / cx, 1.0);
        const double fj = yj * cf;
        y[j] = yj;
        ec[j] = fmax(bj - fj, 0.0);   // >= 0 exactly (y <= 1, z <= 1); clamp rounding
        syf += fj;
        cc = fma(cx - bj, cx - bj, cc);
        const double pj = ((w[j] + wlo[j]) - log(bj)) / sigma;
        psi[j] = pj;
        bg = fma(bj, gamma[j], bg);
        bp = fma(bj, pj, bp);
    }
    syf = wg_red<0>(syf, lds);
    cc = wg_red<0>(cc, lds);
    bg = wg_red<0>(bg, lds);
    bp = wg_red<0>(bp, lds);
    if (threadIdx.x == 0) {
        scal[SC_ER1] = scal[SC_SUMA] - syf;
        scal[SC_COLRES] = cc;
        scal[SC_BG] = bg;
        scal[SC_BP] = bp;
    }
}

// Certificate and KKT finalisation into out[10] (see ibsn_stop in ibsn.h).  ||a||^2 and
// ||b||^2 come from scal[SC_AA], scal[SC_BB].  All the sums are reduced together: one
// shuffle reduction per value in each wave, one exchange through LDS, then thread 0 adds
// the waves' values in wave order.
__global__ __launch_bounds__(NT) void k_stop_final(int G, const double *__restrict__ part,
                                                   const double *__restrict__ rowres_part, int G1,
                                                   double *__restrict__ scal,
                                                   double *__restrict__ out)
{
    constexpr int K = STOP2_NSLOT + 1;   // the stop-pass slots, then the row residual
    __shared__ double lds[K * NW];
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
        v[k] = (k == STOP2_XHMIN) ? INFINITY : 0.0;
    for (int g = threadIdx.x; g < G; g += NT) {
        const double *p = part + (int64_t)g * STOP2_NSLOT;
#pragma unroll
        for (int k = 0; k < STOP2_NSLOT; ++k)
            v[k] = (k == STOP2_XHMIN) ? fmin(v[k], p[k]) : v[k] + p[k];
    }
    for (int g = threadIdx.x; g < G1; g += NT)
        v[STOP2_NSLOT] += rowres_part[g];
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int o = WAVE / 2; o > 0; o >>= 1) {
            const double t = __shfl_xor(v[k], o, WAVE);
            v[k] = (k == STOP2_XHMIN) ? fmin(v[k], t) : v[k] + t;
        }
    }
    const int wv = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            lds[k * NW + wv] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double r = lds[k * NW];
            for (int w = 1; w < NW; ++w)
                r = (k == STOP2_XHMIN) ? fmin(r, lds[k * NW + w]) : r + lds[k * NW + w];
            v[k] = r;
        }
        const double rr = v[STOP2_NSLOT];
        const double na = scal[SC_AA], nb = scal[SC_BB];
        const double dual_g = v[STOP2_AZG] + scal[SC_BG];
        const double dual_p = v[STOP2_AZP] + scal[SC_BP];
        double dp = fmax(sqrt(rr) / (1.0 + sqrt(na)), sqrt(scal[SC_COLRES]) / (1.0 + sqrt(nb)));
        dp = fmax(dp, 0.0 / (1.0 + sqrt(v[STOP2_XF])));
        const double dc = fabs(v[STOP2_XU]) / (1.0 + sqrt(v[STOP2_CF]));
        out[0] = v[STOP2_DPHI];
        out[1] = v[STOP2_CXH];
        out[2] = fmax(dual_g, dual_p);
        out[3] = v[STOP2_CX];
        out[4] = fmax(dp, dc);
        out[5] = v[STOP2_XHMIN];
        out[6] = scal[SC_ER1];
        out[7] = v[STOP2_XU];
        out[8] = dual_g;
        out[9] = dual_p;
    }
}

// outer update of the implicit centre (Algorithm 2, step 13 with eq. (7)):
// r_i = log a_i - (M_i + log S_i); s_j = w_j (= s_j + gamma_j / eta), rounded to one
// double.  The rounding rescales the columns of the new centre X^{k+1} by factors
// 1 + O(2^-53), which the next subproblem's dual absorbs: its optimal plan does not change.
__global__ __launch_bounds__(256) void k_outer_update(int m, int n, const double *__restrict__ a,
                                                      const double *__restrict__ M,
                                                      const double *__restrict__ S,
                                                      const double *__restrict__ w,
                                                      const double *__restrict__ wlo,
                                                      double *__restrict__ r,
                                                      double *__restrict__ s)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < m)
        r[t] = log(a[t]) - (M[t] + log(S[t]));
    if (t < n)
        s[t] = w[t] + wlo[t];
}

// r = log a, s = log b (X^0 = a b^T)
__global__ __launch_bounds__(256) void k_init_center(int m, int n, const double *__restrict__ a,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ r,
                                                     double *__restrict__ s)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < m)
        r[t] = log(a[t]);
    if (t < n)
        s[t] = log(b[t]);
}

// y = alpha x + y (n)
__global__ __launch_bounds__(256) void k_axpy(int n, double alpha, const double *__restrict__ x,
                                              double *__restrict__ y)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n)
        y[j] = fma(alpha, x[j], y[j]);
}

__global__ __launch_bounds__(256) void k_neg(int n, const double *__restrict__ x,
                                             double *__restrict__ y)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n)
        y[j] = -x[j];
}

// Problem checks and per-problem scalars: istar = argmax a (lowest index on ties),
// sum a, sum b, min a, min b, count of non-finite entries of a, b.
__global__ __launch_bounds__(NT) void k_problem_scalars(int m, int n, const double *__restrict__ a,
                                                        const double *__restrict__ b,
                                                        double *__restrict__ scal,
                                                        int *__restrict__ istar)
{
    __shared__ double lds[NW];
    __shared__ int ilds[NT];
    double sa = 0.0, sb = 0.0, mina = INFINITY, minb = INFINITY, bad = 0.0, best = -INFINITY;
    int bi = 0x7fffffff;
    for (int i = threadIdx.x; i < m; i += NT) {
        const double v = a[i];
        sa += v;
        mina = fmin(mina, v);
        if (!isfinite(v))
            bad += 1.0;
        if (v > best) {
            best = v;
            bi = i;
        }
    }
    for (int j = threadIdx.x; j < n; j += NT) {
        const double v = b[j];
        sb += v;
        minb = fmin(minb, v);
        if (!isfinite(v))
            bad += 1.0;
    }
    sa = wg_red<0>(sa, lds);
    sb = wg_red<0>(sb, lds);
    mina = wg_red<2>(mina, lds);
    minb = wg_red<2>(minb, lds);
    bad = wg_red<0>(bad, lds);
    const double gbest = wg_red<1>(best, lds);
    ilds[threadIdx.x] = (best == gbest) ? bi : 0x7fffffff;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            ilds[threadIdx.x] = min(ilds[threadIdx.x], ilds[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scal[SC_SUMA] = sa;
        scal[SC_SUMB] = sb;
        scal[SC_MINA] = mina;
        scal[SC_MINB] = minb;
        scal[SC_BAD] = bad;
        *istar = ilds[0];
        scal[SC_ISTAR] = (double)ilds[0];
    }
}

__global__ __launch_bounds__(256) void k_zero_i32(int64_t count, int32_t *__restrict__ x)
{
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * 256)
        x[t] = 0;
}

}  // namespace

// ---- launchers --------------------------------------------------------------------
#define L1(kern, ...)                                                          \
    do {                                                                       \
        hipLaunchKernelGGL(kern, dim3(1), dim3(NT), 0, st, __VA_ARGS__);       \
        return hipGetLastError();                                              \
    } while (0)

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t sk_gnorms(int64_t n, const double *g, double *scal, hipStream_t st)
{
    L1(k_gnorms, (int)n, g, scal);
}
hipError_t sk_sinkhorn_step(int64_t n, double eta, double q, int split, const double *b,
                            const double *lc, const double *s, double *w, double *wlo,
                            hipStream_t st)
{
    L1(k_sinkhorn_step, (int)n, eta, q, split, b, lc, s, w, wlo);
}
hipError_t sk_dd_axpy(int64_t n, double q, const double *d, double *w, double *wlo, hipStream_t st)
{
    hipLaunchKernelGGL(k_dd_axpy, dim3(nblk(n)), dim3(256), 0, st, (int)n, q, d, w, wlo);
    return hipGetLastError();
}
hipError_t sk_log(int64_t n, const double *c, double *lc, hipStream_t st)
{
    hipLaunchKernelGGL(k_log, dim3(nblk(n)), dim3(256), 0, st, (int)n, c, lc);
    return hipGetLastError();
}
hipError_t sk_wmax(int64_t n, const double *s, const double *gamma, double eta, double *scal,
                   hipStream_t st)
{
    L1(k_wmax, (int)n, s, gamma, eta, scal);
}
hipError_t sk_cost_max(int64_t m, int64_t n, int64_t ldc, int kind, const void *C,
                       const double *py, double pscale, double *part, int G, double *scal,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_cost_max_part, dim3(G), dim3(256), 0, st, (int)m, (int)n, ldc, kind, C,
                       py, pscale, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(NT), 0, st, G, 1, 0, part, 1.0, 0.0, -1, SC_CMAX,
                       1, scal);
    return hipGetLastError();
}
hipError_t sk_gamma_of(int64_t n, double eta, const double *w, const double *wlo, const double *s,
                       double *gamma, hipStream_t st)
{
    hipLaunchKernelGGL(k_gamma_of, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (int)n, eta,
                       w, wlo, s, gamma);
    return hipGetLastError();
}
hipError_t sk_center(int64_t n, double *gamma, hipStream_t st) { L1(k_center, (int)n, gamma); }
hipError_t sk_trial_prep(int64_t n, double t, double eta, double q, int split, const double *Delta,
                         const double *b, double *tau, double *colv, double *scal, hipStream_t st)
{
    L1(k_trial_prep, (int)n, t, eta, q, split, Delta, b, tau, colv, scal);
}
hipError_t sk_sum_parts(int G, int stride, int off, const double *part, double alpha, double beta,
                        int src, int slot, int op, double *scal, hipStream_t st)
{
    L1(k_sum_parts, G, stride, off, part, alpha, beta, src, slot, op, scal);
}
hipError_t sk_dot_slot(int64_t n, const double *x, const double *y, int slot, double *scal,
                       hipStream_t st)
{
    L1(k_dot_slot, (int)n, x, y, slot, scal);
}
hipError_t sk_stop_prep(int64_t n, double sigma, const double *b, const double *w,
                        const double *wlo, const double *gamma, const double *colX,
                        const double *colF, double *y, double *ec, double *psi, double *scal,
                        hipStream_t st)
{
    L1(k_stop_prep, (int)n, sigma, b, w, wlo, gamma, colX, colF, y, ec, psi, scal);
}
hipError_t sk_fill(int64_t n, double v, double *x, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(256), 0, st, (int)n, v, x);
    return hipGetLastError();
}
hipError_t sk_stop_final(int G, const double *part, const double *rowres_part, int G1,
                         double *scal, double *out, hipStream_t st)
{
    L1(k_stop_final, G, part, rowres_part, G1, scal, out);
}
hipError_t sk_problem_scalars(int64_t m, int64_t n, const double *a, const double *b,
                              double *scal, int *istar, hipStream_t st)
{
    L1(k_problem_scalars, (int)m, (int)n, a, b, scal, istar);
}
hipError_t sk_outer_update(int64_t m, int64_t n, const double *a, const double *M, const double *S,
                           const double *w, const double *wlo, double *r, double *s, hipStream_t st)
{
    hipLaunchKernelGGL(k_outer_update, dim3(nblk(m > n ? m : n)), dim3(256), 0, st, (int)m, (int)n,
                       a, M, S, w, wlo, r, s);
    return hipGetLastError();
}
hipError_t sk_init_center(int64_t m, int64_t n, const double *a, const double *b, double *r,
                          double *s, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_center, dim3(nblk(m > n ? m : n)), dim3(256), 0, st, (int)m, (int)n,
                       a, b, r, s);
    return hipGetLastError();
}
hipError_t sk_axpy(int64_t n, double alpha, const double *x, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_axpy, dim3(nblk(n)), dim3(256), 0, st, (int)n, alpha, x, y);
    return hipGetLastError();
}
hipError_t sk_neg(int64_t n, const double *x, double *y, hipStream_t st)
{
    hipLaunchKernelGGL(k_neg, dim3(nblk(n)), dim3(256), 0, st, (int)n, x, y);
    return hipGetLastError();
}
hipError_t sk_zero_i32(int64_t count, int32_t *x, hipStream_t st)
{
    int64_t b = (count + 255) / 256;
    if (b > 4096)
        b = 4096;
    if (b < 1)
        b = 1;
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)b), dim3(256), 0, st, count, x);
    return hipGetLastError();
}

}  // namespace ibsn
