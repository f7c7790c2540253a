// dense_collse.hip -- column log-sum-exp pass for the Sinkhorn gamma-step in the log domain,
// on gfx950; helpers in dense_common.h.
//
// The Sinkhorn step of the warm-up (Algorithm 2, steps 3-4) moves w_j by log b_j - log c_j,
// c_j = sum_i a_i P_ij the column sums of the eval pass.  At small eta (large sigma) every
// kernel entry of a column can lie below the FP64 range, c_j = 0 and log c_j = -inf.  This
// pass forms log c_j directly as
//     lc_j = LSE_i (x_ij + log a_i - log S_i),   x_ij = theta_ij - M_i,
// with a running maximum per column, so lc_j is finite whatever the scale of the column.
//
// Layout: one thread per column (consecutive threads read consecutive columns of a row, a
// coalesced read of the row-major cost), a grid of column blocks x row blocks; each thread
// keeps an online pair (m, s) with sum = s e^m over its row block.  A second kernel combines
// the row blocks' pairs per column in row-block order, so the result is reproducible.
#include "dense_common.h"

namespace ibsn {
namespace {

constexpr int CL_NT = 256;   // threads (columns) per workgroup
constexpr int CL_RC = 256;   // rows of per-row scalars staged per chunk

template <typename CT>
struct ColCost {
    __device__ __forceinline__ ColCost(const void *, const double *, double, int) {}
    __device__ __forceinline__ double at(const void *C, int64_t ldc, int i, int j) const
    {
        return (double)static_cast<const CT *>(C)[(int64_t)i * ldc + j];
    }
};
template <int DIM>
struct ColCost<PtsCost<DIM>> {
    double yj[DIM];
    double scale;
    __device__ __forceinline__ ColCost(const void *, const double *py, double s, int j) : scale(s)
    {
#pragma unroll
        for (int k = 0; k < DIM; ++k)
            yj[k] = py[(int64_t)j * DIM + k];
    }
    __device__ __forceinline__ double at(const void *C, int64_t, int i, int) const
    {
        const double *x = static_cast<const double *>(C) + (int64_t)i * DIM;
        double xi[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k)
            xi[k] = x[k];
        return pts_cost<DIM>(xi, yj, scale);
    }
};

template <typename CT, bool LO>
__global__ __launch_bounds__(CL_NT) void k_collse_part(const void *__restrict__ C, int64_t ldc,
                                                       const double *__restrict__ py,
                                                       double pscale, int m, int n, int RB,
                                                       double sigma, const double *__restrict__ w,
                                                       const double *__restrict__ wlo,
                                                       const double *__restrict__ a,
                                                       const double *__restrict__ M,
                                                       const double *__restrict__ S,
                                                       double *__restrict__ pmax,
                                                       double *__restrict__ psum)
{
    __shared__ double etab[EXP_TAB];
    __shared__ double rM[CL_RC], rR[CL_RC];
    exp_table_init(etab);
    const int rb = blockIdx.y;
    const int i0 = (int)((int64_t)m * rb / RB), i1 = (int)((int64_t)m * (rb + 1) / RB);
    const int j = blockIdx.x * CL_NT + threadIdx.x;
    const int jc = j < n ? j : n - 1;   // threads past n read column n - 1 and store nothing
    const ColCost<CT> cost(C, py, pscale, jc);
    const double wh = w[jc];
    const double wl = LO ? wlo[jc] : 0.0;
    double mx = -INFINITY, sm = 0.0;
    for (int c0 = i0; c0 < i1; c0 += CL_RC) {
        const int cnt = min(CL_RC, i1 - c0);
        __syncthreads();   // the previous chunk may still be read
        for (int r = threadIdx.x; r < cnt; r += CL_NT) {
            rM[r] = M[c0 + r];
            rR[r] = log(a[c0 + r]) - log(S[c0 + r]);
        }
        __syncthreads();
        for (int r = 0; r < cnt; ++r) {
            double x = fma(-sigma, cost.at(C, ldc, c0 + r, jc), wh - rM[r]);
            if constexpr (LO)
                x += wl;
            const double v = x + rR[r];
            // online LSE: sum = sm e^mx; a larger v rescales the sum to its own shift
            const double d = v - mx;
            const double e = exp_tab(-fabs(d), etab);
            sm = d > 0.0 ? fma(sm, e, 1.0) : sm + e;
            mx = fmax(mx, v);
        }
    }
    if (j < n) {
        pmax[(int64_t)rb * n + j] = mx;
        psum[(int64_t)rb * n + j] = sm;
    }
}

__global__ __launch_bounds__(256) void k_collse_combine(int n, int RB,
                                                        const double *__restrict__ pmax,
                                                        const double *__restrict__ psum,
                                                        double *__restrict__ lc)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n)
        return;
    double M = -INFINITY;
    for (int rb = 0; rb < RB; ++rb)
        M = fmax(M, pmax[(int64_t)rb * n + j]);
    double s = 0.0;
    for (int rb = 0; rb < RB; ++rb)
        s += psum[(int64_t)rb * n + j] * exp(pmax[(int64_t)rb * n + j] - M);
    lc[j] = M + log(s);
}

}  // namespace

int collse_row_blocks(int64_t m, int64_t n, int max_rb)
{
    const int64_t cb = (n + CL_NT - 1) / CL_NT;
    int64_t rb = (1024 + cb - 1) / cb;   // about 1024 workgroups
    rb = rb < m ? rb : m;
    rb = rb < max_rb ? rb : max_rb;
    return (int)(rb > 0 ? rb : 1);
}

hipError_t launch_collse(const DenseArgs &d, int lo, const double *M, const double *S, int RB,
                         double *pmax, double *psum, double *lc, hipStream_t st)
{
    const dim3 grid((unsigned)((d.n + CL_NT - 1) / CL_NT), (unsigned)RB);
#define COLLSE(CTT)                                                                              \
    do {                                                                                         \
        if (lo)                                                                                  \
            hipLaunchKernelGGL((k_collse_part<CTT, true>), grid, dim3(CL_NT), 0, st, d.C, d.ldc, \
                               d.py, d.pscale, (int)d.m, (int)d.n, RB, d.sigma, d.w, d.wlo, d.a, \
                               M, S, pmax, psum);                                                \
        else                                                                                     \
            hipLaunchKernelGGL((k_collse_part<CTT, false>), grid, dim3(CL_NT), 0, st, d.C,       \
                               d.ldc, d.py, d.pscale, (int)d.m, (int)d.n, RB, d.sigma, d.w,      \
                               d.wlo, d.a, M, S, pmax, psum);                                    \
    } while (0)
    if (d.cost_kind == 0)
        COLLSE(double);
    else if (d.cost_kind == 1)
        COLLSE(float);
    else if (d.pdim == 2)
        COLLSE(PtsCost<2>);
    else
        COLLSE(PtsCost<3>);
#undef COLLSE
    hipLaunchKernelGGL(k_collse_combine, dim3((unsigned)((d.n + 255) / 256)), dim3(256), 0, st,
                       (int)d.n, RB, pmax, psum, lc);
    return hipGetLastError();
}

}  // namespace ibsn
