// warmstart.hip -- learned warm start for the first proximal subproblem's dual, on gfx950.
//
// Algorithm 2 starts from gamma^{0,0} = 0.  This module predicts a starting dual instead:
// a point-set network reads the two point clouds and predicts, for every target point,
// the dual of the first subproblem (zero initialisation stays the fallback).
//
// Network (widths 256, ReLU):
//   encoder   per point p (sources and targets alike), features f_p in R^4,
//             e_p = W3 relu(W2 relu(W1 f_p + b1) + b2) + b3                    (3 layers)
//   pooling   h_s = mean over the sources of e_p, h_t = mean over the targets, and the
//             instance's context c = Wc [h_s; h_t] + bc
//   head      per target j, features u_j in R^8,
//             z1 = relu(Wf u_j + bf),  z2 = relu(Wg z1 + bg),
//             o_j = z2 . c + ws . u_j + bo                                     (3 layers)
//   output    gamma_j = scale (o_j - mean_j o_j)   (the subproblem's dual is defined up
//             to a constant; scale = u s below, the unit in which the first subproblem's
//             dual varies at every size)
// Features: sources (x~_i1, x~_i2, m a_i, +1), targets (y~_j1, y~_j2, n b_j, -1) for the
// encoder in box coordinates; for the head (y~_j1, y~_j2, n b_j, min_i C_ij / mean cmin)
// and four potentials G_k of the linearised Monge-Ampere equation (the Laplacian of the
// dual's potential is the difference of the two densities to first order), smoothed at
// four lengths, with mirror images for the box.  At small eta the first subproblem's dual
// is close to the optimal transport potential, and these four values alone carry most of
// its variance; the network learns their combination and the rest.
//
// Arithmetic: every matrix product is a BF16 MFMA (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation; its operands are rounded to BF16 (round to nearest even) where they enter
// a product: the weights (BF16 copies of FP32 master weights), the layer inputs and, in the
// backward pass, the output gradients.  Biases, activations, pooling, the linear path, the
// loss and the Adam update are FP32.
#include "../../include/ibsn.h"
#include "ibsn_internal.h"

#include <math.h>

#include <cstring>
#include <random>
#include <vector>

using namespace ibsn;

#define CKI(call)                  \
    do {                           \
        const int rc_ = (call);    \
        if (rc_ < 0)               \
            return rc_;            \
    } while (0)

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int WID = 256;   // width of every hidden layer
constexpr int NF = 4;      // encoder features per point
constexpr int NFH = 8;     // head features per target

// ---------------------------------------------------------------------------------
// C = act(A B + bias + rowbias[row / grp]) for A (M x K), B (K x N) in BF16 with general
// strides (A_ik = A[i sar + k sac], B_kj = B[k sbr + j sbc]), FP32 accumulation.
// Block tile 64 x 64 (four waves, each 32 x 32 = 2 x 2 MFMA tiles of 16 x 16), K in steps
// of 32 staged in LDS as As[row][k] and Bs[col][k], so that each lane's 8 consecutive k
// values are one 16-byte LDS read.  MFMA 16x16x32 operand layout: lane l holds
// A[l % 16][8 (l / 16) .. +7] and B[8 (l / 16) .. +7][l % 16]; the result lane l holds
// D[4 (l / 16) + i][l % 16], i < 4.  Out-of-range rows, columns and k are zero in LDS.
// Outputs: C32 (FP32) and / or C16 (BF16), leading dimension ldc; either may be null.
// ---------------------------------------------------------------------------------
template <bool RELU>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const bf16 *__restrict__ A,
                                              int64_t sar, int64_t sac, const bf16 *__restrict__ B,
                                              int64_t sbr, int64_t sbc,
                                              const float *__restrict__ bias,
                                              const float *__restrict__ rowbias, int grp,
                                              float *__restrict__ C32, bf16 *__restrict__ C16,
                                              int ldc)
{
    constexpr int LDK = 40;   // 32 + 8: rows of 80 bytes, 16-byte aligned
    __shared__ __align__(16) bf16 As[64][LDK];
    __shared__ __align__(16) bf16 Bs[64][LDK];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv >> 1, wn = wv & 1;
    const int row0 = blockIdx.y * 64, col0 = blockIdx.x * 64;
    floatx4 acc[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
            acc[ti][tj] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bf16 zero = (bf16)0.0f;
    for (int k0 = 0; k0 < K; k0 += 32) {
        // consecutive threads take consecutive addresses where the strides allow: A with
        // k fastest when its k stride is 1 (rows fastest otherwise), B with columns fastest
        // when its column stride is 1 (k fastest otherwise)
        for (int e = tid; e < 64 * 32; e += 256) {
            const int r = sac == 1 ? (e >> 5) : (e & 63), kk = sac == 1 ? (e & 31) : (e >> 6);
            const int gi = row0 + r, gk = k0 + kk;
            As[r][kk] = (gi < M && gk < K) ? A[gi * sar + gk * sac] : zero;
            const int kb = sbc == 1 ? (e >> 6) : (e & 31), c = sbc == 1 ? (e & 63) : (e >> 5);
            const int gj = col0 + c, gkb = k0 + kb;
            Bs[c][kb] = (gj < N && gkb < K) ? B[gkb * sbr + gj * sbc] : zero;
        }
        __syncthreads();
#pragma unroll
        for (int ti = 0; ti < 2; ++ti) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(
                &As[wm * 32 + ti * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
            for (int tj = 0; tj < 2; ++tj) {
                const bf16x8 b = *reinterpret_cast<const bf16x8 *>(
                    &Bs[wn * 32 + tj * 16 + (lane & 15)][8 * (lane >> 4)]);
                acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[ti][tj], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
            const int col = col0 + wn * 32 + tj * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = row0 + wm * 32 + ti * 16 + 4 * (lane >> 4) + i;
                if (row < M && col < N) {
                    float v = acc[ti][tj][i];
                    if (bias)
                        v += bias[col];
                    if (rowbias)
                        v += rowbias[(int64_t)(row / grp) * N + col];
                    if (RELU)
                        v = fmaxf(v, 0.0f);
                    if (C32)
                        C32[(int64_t)row * ldc + col] = v;
                    if (C16)
                        C16[(int64_t)row * ldc + col] = (bf16)v;
                }
            }
        }
}

__global__ void k_to_bf16(int64_t n, const float *__restrict__ x, bf16 *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        y[i] = (bf16)x[i];
}

// dZ (in place) *= (Z > 0) for a ReLU output Z; BF16 copy of the result
__global__ void k_relu_bwd(int64_t n, float *__restrict__ dz, const float *__restrict__ z,
                           bf16 *__restrict__ dz16)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const float v = z[i] > 0.0f ? dz[i] : 0.0f;
        dz[i] = v;
        dz16[i] = (bf16)v;
    }
}

// out[g][c] = alpha * sum over rows r of group g (rows g*rows .. +rows-1) of X[r][c] (+ beta
// out[g][c] when accumulate): one thread per (group, column), rows in order.
__global__ void k_group_sum(int G, int rows, int N, const float *__restrict__ X, float alpha,
                            int accumulate, float *__restrict__ out)
{
    const int c = blockIdx.x * 256 + threadIdx.x, g = blockIdx.y;
    if (c >= N)
        return;
    const float *x = X + (int64_t)g * rows * N + c;
    float s = 0.0f;
    for (int r = 0; r < rows; ++r)
        s += x[(int64_t)r * N];
    out[(int64_t)g * N + c] = accumulate ? out[(int64_t)g * N + c] + alpha * s : alpha * s;
}

// dX[r][c] = alpha * dOut[(r / rows) * ld + c] (the backward pass of a group mean; rows of
// dX are R x N, row-major)
__global__ void k_group_bcast(int64_t R, int rows, int N, const float *__restrict__ dout,
                              int64_t ld, float alpha, float *__restrict__ dx)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < R * N) {
        const int64_t r = i / N;
        const int c = (int)(i % N);
        dx[i] = alpha * dout[(r / rows) * ld + c];
    }
}

// per instance b (n outputs o): centred output oc = o - mean o; loss partial
// sum (oc - t)^2; gradient d o_j = (2 / (B n)) ((oc_j - t_j) - mean_j (oc - t)).
// One workgroup per instance.
__global__ __launch_bounds__(256) void k_head_loss(int n, const float *__restrict__ o,
                                                   const float *__restrict__ t, float inv_total,
                                                   float *__restrict__ loss_part,
                                                   float *__restrict__ dout)
{
    __shared__ float red[256];
    const int b = blockIdx.x;
    const float *ob = o + (int64_t)b * n, *tb = t + (int64_t)b * n;
    float s = 0.0f;
    for (int j = threadIdx.x; j < n; j += 256)
        s += ob[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const float mo = red[0] / (float)n;
    __syncthreads();
    float l = 0.0f, sd = 0.0f;
    for (int j = threadIdx.x; j < n; j += 256) {
        const float d = (ob[j] - mo) - tb[j];
        l += d * d;
        sd += d;
    }
    red[threadIdx.x] = sd;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const float md = red[0] / (float)n;
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += 256)
        dout[(int64_t)b * n + j] = 2.0f * inv_total * (((ob[j] - mo) - tb[j]) - md);
    red[threadIdx.x] = l;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        loss_part[b] = red[0];
}

// Adam (Kingma and Ba, 2015) on the FP32 master weights, with the BF16 copy refreshed
__global__ void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g,
                       float *__restrict__ m1, float *__restrict__ m2, bf16 *__restrict__ p16,
                       float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const float gi = g[i];
        const float a = b1 * m1[i] + (1.0f - b1) * gi;
        const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
        m1[i] = a;
        m2[i] = v;
        const float np = p[i] - lr * (a / c1) / (sqrtf(v / c2) + eps);
        p[i] = np;
        if (p16)
            p16[i] = (bf16)np;
    }
}

// gamma_j = scale (o_j - mean o) for one instance (double output), one workgroup
__global__ __launch_bounds__(256) void k_predict_out(int n, const float *__restrict__ o,
                                                     double scale, double *__restrict__ gamma)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += 256)
        s += (double)o[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double mo = red[0] / (double)n;
    for (int j = threadIdx.x; j < n; j += 256)
        gamma[j] = scale * ((double)o[j] - mo);
}

// min_i C_ij per column (a thread per column, rows in order)
template <typename CT>
__global__ void k_colmin(int m, int n, const CT *__restrict__ C, int64_t ldc,
                         double *__restrict__ out)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n)
        return;
    double v = INFINITY;
    for (int i = 0; i < m; ++i)
        v = fmin(v, (double)C[(int64_t)i * ldc + j]);
    out[j] = v;
}
__global__ void k_colmin_pts(int m, int n, int dim, const double *__restrict__ x,
                             const double *__restrict__ y, double scale, double *__restrict__ out)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n)
        return;
    double v = INFINITY;
    for (int i = 0; i < m; ++i) {
        double s = 0.0;
        for (int k = 0; k < dim; ++k) {
            const double t = x[(int64_t)i * dim + k] - y[(int64_t)j * dim + k];
            s = k == 0 ? t * t : s + t * t;
        }
        v = fmin(v, s * scale);
    }
    out[j] = v;
}

// ol_t = sum_k ws_k f_tk (FP32, k in order)
__global__ void k_lin_fwd(int64_t T, const float *__restrict__ f, const float *__restrict__ ws,
                          float *__restrict__ ol)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= T)
        return;
    float v = 0.0f;
#pragma unroll
    for (int k = 0; k < NFH; ++k)
        v = fmaf(ws[k], f[t * NFH + k], v);
    ol[t] = v;
}

// gws_k = sum_t dO_t f_tk, one workgroup per k (fixed order)
__global__ __launch_bounds__(256) void k_lin_grad(int64_t T, const float *__restrict__ f,
                                                  const float *__restrict__ dO,
                                                  float *__restrict__ gws)
{
    __shared__ float red[256];
    const int k = blockIdx.x;
    float s = 0.0f;
    for (int64_t t = threadIdx.x; t < T; t += 256)
        s = fmaf(dO[t], f[t * NFH + k], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        gws[k] = red[0];
}

// mean of an n-vector into out[0] (one workgroup)
__global__ __launch_bounds__(256) void k_mean(int n, const double *__restrict__ x,
                                              double *__restrict__ out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += 256)
        s += x[j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[0] = red[0] / (double)n;
}

// ---- features -----------------------------------------------------------------
// Coordinates are taken in the bounding box of all points (shifted to the origin, divided
// by its longer side L); u = kappa L^2 is the cost of a unit box distance squared (kappa =
// C_ii / |x_i - y_i|^2 summed over the first K pairs, or the points cost's own scale) and
// s = sqrt(mean_j min_i C_ij / u) the typical nearest-source distance in box units.
// par: [0] lo1 [1] lo2 [2] L [3] hin1 [4] hin2 [5] kappa [6] u [7] mean cmin [8] s
//      [9..12] mean_j G_k
enum { PR_LO1, PR_LO2, PR_L, PR_HI1, PR_HI2, PR_KAPPA, PR_U, PR_CMEAN, PR_S, PR_GM, PR_N = 16 };
constexpr int KAPPA_PAIRS = 4096;
constexpr int NGREEN = 4;
__constant__ float GREEN_EPS2[NGREEN] = {1e-4f, 4e-4f, 1.6e-3f, 6.4e-3f};   // (0.01 .. 0.08)^2

__device__ __forceinline__ double blk_red(double v, double *red, int op)   // 0 sum 1 min 2 max
{
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double o = red[threadIdx.x + w], c = red[threadIdx.x];
            red[threadIdx.x] = op == 0 ? c + o : (op == 1 ? fmin(c, o) : fmax(c, o));
        }
        __syncthreads();
    }
    return red[0];
}

// box, kappa, u (one workgroup of 1024 threads)
template <typename CT>
__global__ __launch_bounds__(1024) void k_box(int m, int n, const double *__restrict__ x,
                                              const double *__restrict__ y, const CT *C,
                                              int64_t ldc, double pts_scale,
                                              double *__restrict__ par)
{
    __shared__ double red[1024];
    double mn[2] = {INFINITY, INFINITY}, mx[2] = {-INFINITY, -INFINITY};
    for (int t = threadIdx.x; t < m + n; t += 1024) {
        const double *q = t < m ? x + 2 * (int64_t)t : y + 2 * (int64_t)(t - m);
        for (int d = 0; d < 2; ++d) {
            mn[d] = fmin(mn[d], q[d]);
            mx[d] = fmax(mx[d], q[d]);
        }
    }
    const int K = min(min(m, n), KAPPA_PAIRS);
    double num = 0.0, den = 0.0;
    for (int i = threadIdx.x; i < K; i += 1024) {
        const double d0 = x[2 * i] - y[2 * i], d1 = x[2 * i + 1] - y[2 * i + 1];
        den += d0 * d0 + d1 * d1;
        if (C)
            num += (double)C[(int64_t)i * ldc + i];
    }
    const double lo1 = blk_red(mn[0], red, 1), lo2 = blk_red(mn[1], red, 1);
    const double hi1 = blk_red(mx[0], red, 2), hi2 = blk_red(mx[1], red, 2);
    num = blk_red(num, red, 0);
    den = blk_red(den, red, 0);
    if (threadIdx.x == 0) {
        double L = fmax(hi1 - lo1, hi2 - lo2);
        L = L > 0.0 ? L : 1.0;
        const double kappa = C ? (den > 0.0 ? num / den : 1.0) : pts_scale;
        par[PR_LO1] = lo1;
        par[PR_LO2] = lo2;
        par[PR_L] = L;
        par[PR_HI1] = (hi1 - lo1) / L;
        par[PR_HI2] = (hi2 - lo2) / L;
        par[PR_KAPPA] = kappa;
        par[PR_U] = kappa * L * L;
    }
}

// Potentials of the linearised Monge-Ampere equation:
//   G_k(j) = sum_i a_i g_k(x_i, y_j) - sum_l b_l g_k(y_l, y_j),
//   g_k(p, q) = log(|p - q|^2 + eps_k^2) / 2 summed over the nine mirror images of p in the
// box (a reflecting boundary).  Grid (target blocks, point splits): thread j of split sp
// adds the points [q0, q1) of the combined list (sources, then targets with weight -b),
// staged 256 at a time in LDS as FP32 box coordinates; logs in FP32 (log2, scaled at the
// end), each tile's sum in FP32, the tiles' sums in FP64.  gpart[sp][j][k].
__global__ __launch_bounds__(256) void k_green(int m, int n, int per, const double *__restrict__ x,
                                               const double *__restrict__ y,
                                               const double *__restrict__ a,
                                               const double *__restrict__ b,
                                               const double *__restrict__ par,
                                               double *__restrict__ gpart)
{
    __shared__ float px[256], py[256], pw[256];
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int sp = blockIdx.y;
    const int q0 = sp * per, q1 = min(m + n, q0 + per);
    const double lo1 = par[PR_LO1], lo2 = par[PR_LO2], iL = 1.0 / par[PR_L];
    const float h1 = (float)(2.0 * par[PR_HI1]), h2 = (float)(2.0 * par[PR_HI2]);
    const int jc = j < n ? j : n - 1;
    const float yj1 = (float)((y[2 * (int64_t)jc] - lo1) * iL);
    const float yj2 = (float)((y[2 * (int64_t)jc + 1] - lo2) * iL);
    double acc[NGREEN] = {0.0, 0.0, 0.0, 0.0};
    for (int t0 = q0; t0 < q1; t0 += 256) {
        __syncthreads();
        {
            const int q = t0 + threadIdx.x;
            float u1 = 0.0f, u2 = 0.0f, w = 0.0f;
            if (q < q1) {
                const double *pt = q < m ? x + 2 * (int64_t)q : y + 2 * (int64_t)(q - m);
                u1 = (float)((pt[0] - lo1) * iL);
                u2 = (float)((pt[1] - lo2) * iL);
                w = q < m ? (float)a[q] : -(float)b[q - m];
            }
            px[threadIdx.x] = u1;
            py[threadIdx.x] = u2;
            pw[threadIdx.x] = w;
        }
        __syncthreads();
        const int cnt = min(256, q1 - t0);
        float s[NGREEN] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int e = 0; e < cnt; ++e) {
            const float p1 = px[e], p2 = py[e], w = pw[e];
            const float ix[3] = {-p1 - yj1, p1 - yj1, h1 - p1 - yj1};
            const float iy[3] = {-p2 - yj2, p2 - yj2, h2 - p2 - yj2};
            float l[NGREEN] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int u = 0; u < 3; ++u)
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    const float D = fmaf(ix[u], ix[u], iy[v] * iy[v]);
#pragma unroll
                    for (int k = 0; k < NGREEN; ++k)
                        l[k] += __log2f(D + GREEN_EPS2[k]);
                }
#pragma unroll
            for (int k = 0; k < NGREEN; ++k)
                s[k] = fmaf(w, l[k], s[k]);
        }
#pragma unroll
        for (int k = 0; k < NGREEN; ++k)
            acc[k] += (double)s[k];
    }
    if (j < n) {
        constexpr double HALF_LN2 = 0.34657359027997264;   // log(2) / 2
#pragma unroll
        for (int k = 0; k < NGREEN; ++k)
            gpart[((int64_t)sp * n + j) * NGREEN + k] = acc[k] * HALF_LN2;
    }
}

// G (n x 4) = sum of the splits in order
__global__ void k_green_sum(int n, int splits, const double *__restrict__ gpart,
                            double *__restrict__ g)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n)
        return;
    for (int k = 0; k < NGREEN; ++k) {
        double v = 0.0;
        for (int sp = 0; sp < splits; ++sp)
            v += gpart[((int64_t)sp * n + j) * NGREEN + k];
        g[(int64_t)j * NGREEN + k] = v;
    }
}

// means of cmin and of the G columns, and s (one workgroup of 1024 threads)
__global__ __launch_bounds__(1024) void k_feat_means(int n, const double *__restrict__ cmin,
                                                     const double *__restrict__ g,
                                                     double *__restrict__ par)
{
    __shared__ double red[1024];
    double c = 0.0, gs[NGREEN] = {0.0, 0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < n; j += 1024) {
        c += cmin[j];
        for (int k = 0; k < NGREEN; ++k)
            gs[k] += g[(int64_t)j * NGREEN + k];
    }
    const double cm = blk_red(c, red, 0) / (double)n;
    double gm[NGREEN];
    for (int k = 0; k < NGREEN; ++k)
        gm[k] = blk_red(gs[k], red, 0) / (double)n;
    if (threadIdx.x == 0) {
        const double u = par[PR_U];
        par[PR_CMEAN] = cm;
        par[PR_S] = u > 0.0 ? sqrt(fmax(cm / u, 1e-12)) : 1.0;
        for (int k = 0; k < NGREEN; ++k)
            par[PR_GM + k] = gm[k];
    }
}

// fs (m x 4) = (x~1, x~2, m a, +1); fte (n x 4) = (y~1, y~2, n b, -1);
// fth (n x 8) = (y~1, y~2, n b, cmin / mean cmin, (G_k - mean G_k) / s)
__global__ void k_features(int m, int n, const double *__restrict__ x,
                           const double *__restrict__ y, const double *__restrict__ a,
                           const double *__restrict__ b, const double *__restrict__ cmin,
                           const double *__restrict__ g, const double *__restrict__ par,
                           float *__restrict__ fs, float *__restrict__ fte,
                           float *__restrict__ fth)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    const double lo1 = par[PR_LO1], lo2 = par[PR_LO2], iL = 1.0 / par[PR_L];
    if (t < m) {
        fs[4 * t + 0] = (float)((x[2 * t] - lo1) * iL);
        fs[4 * t + 1] = (float)((x[2 * t + 1] - lo2) * iL);
        fs[4 * t + 2] = (float)((double)m * a[t]);
        fs[4 * t + 3] = 1.0f;
    }
    if (t < n) {
        const float y0 = (float)((y[2 * t] - lo1) * iL), y1 = (float)((y[2 * t + 1] - lo2) * iL);
        const float w = (float)((double)n * b[t]);
        fte[4 * t + 0] = y0;
        fte[4 * t + 1] = y1;
        fte[4 * t + 2] = w;
        fte[4 * t + 3] = -1.0f;
        float *h = fth + (int64_t)NFH * t;
        h[0] = y0;
        h[1] = y1;
        h[2] = w;
        h[3] = (float)(cmin[t] / par[PR_CMEAN]);
        const double is = 1.0 / par[PR_S];
        for (int k = 0; k < NGREEN; ++k)
            h[4 + k] = (float)((g[(int64_t)t * NGREEN + k] - par[PR_GM + k]) * is);
    }
}

unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// ---------------------------------------------------------------------------------
// the model: parameters in a fixed order (W1 b1 W2 b2 W3 b3 Wf bf Wg bg Wc bc ws bo; a weight
// matrix is inputs x outputs, row-major), FP32 master copies, BF16 copies, Adam moments,
// gradients, and grow-only activation buffers
// ---------------------------------------------------------------------------------
namespace {
struct Param {
    int rows, cols;
    int64_t off;
};
constexpr int NPARAM = 14;
enum { P_W1, P_B1, P_W2, P_B2, P_W3, P_B3, P_WF, P_BF, P_WG, P_BG, P_WC, P_BC, P_WS, P_BO };
const int SHAPES[NPARAM][2] = {{NF, WID},  {1, WID},  {WID, WID}, {1, WID},      {WID, WID},
                               {1, WID},   {NFH, WID}, {1, WID},  {WID, WID},    {1, WID},
                               {2 * WID, WID}, {1, WID}, {NFH, 1},  {1, 1}};
int64_t layout(Param *p)
{
    int64_t off = 0;
    for (int i = 0; i < NPARAM; ++i) {
        p[i] = Param{SHAPES[i][0], SHAPES[i][1], off};
        off += (int64_t)SHAPES[i][0] * SHAPES[i][1];
    }
    return off;
}

template <typename T>
struct Buf {
    T *p = nullptr;
    size_t n = 0;
    bool ensure(size_t cnt)
    {
        if (cnt <= n)
            return true;
        release();
        if (hipMalloc(&p, cnt * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return false;
        }
        n = cnt;
        return true;
    }
    void release()
    {
        if (p)
            (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// activations (FP32 and BF16) and their gradients
enum { A_X, A_XH, A_H1, A_H2, A_E, A_CTX, A_CB, A_Z1, A_Z2, A_O, A_OL, A_TMP, A_N };
}  // namespace

struct ibsn_ws_model {
    ibsn_ctx *ctx = nullptr;
    Param prm[NPARAM];
    int64_t total = 0;
    Buf<float> w, g, m1, m2, part;
    Buf<bf16> w16;
    int64_t step = 0;
    Buf<float> a32[A_N], d32[A_N];
    Buf<bf16> a16[A_N], d16[A_N];
};

namespace {

#define WCK(call)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ctx_fail(ctx, IBSN_ERR_HIP, hipGetErrorString(e_));                   \
    } while (0)
#define WNEED(buf, cnt)                                                                  \
    do {                                                                                 \
        if (!(buf).ensure((size_t)(cnt)))                                                \
            return ctx_fail(ctx, IBSN_ERR_OOM, "warm-start buffers: out of memory");     \
    } while (0)

hipError_t gemm(hipStream_t st, bool relu, int64_t M, int64_t N, int64_t K, const bf16 *A,
                int64_t sar, int64_t sac, const bf16 *B, int64_t sbr, int64_t sbc,
                const float *bias, const float *rowbias, int64_t grp, float *C32, bf16 *C16,
                int64_t ldc)
{
    const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
    if (relu)
        hipLaunchKernelGGL(k_gemm<true>, grid, dim3(256), 0, st, (int)M, (int)N, (int)K, A, sar,
                           sac, B, sbr, sbc, bias, rowbias, (int)grp, C32, C16, (int)ldc);
    else
        hipLaunchKernelGGL(k_gemm<false>, grid, dim3(256), 0, st, (int)M, (int)N, (int)K, A, sar,
                           sac, B, sbr, sbc, bias, rowbias, (int)grp, C32, C16, (int)ldc);
    return hipGetLastError();
}

// column sums of X (rows x N) into out (N), in row order per column
hipError_t colsum(hipStream_t st, int64_t rows, int64_t N, const float *X, float *out)
{
    hipLaunchKernelGGL(k_group_sum, dim3((unsigned)((N + 255) / 256), 1), dim3(256), 0, st, 1,
                       (int)rows, (int)N, X, 1.0f, 0, out);
    return hipGetLastError();
}

// Forward pass for B instances of m sources and n targets.  The encoder runs over the
// stacked points: rows [0, B m) are the sources (instance b at b m ..), rows [B m, B (m+n))
// the targets.  Keeps H1, H2, Z1, Z2 (FP32, BF16), E (FP32), CTX (FP32, BF16), O (FP32).
int forward(ibsn_ctx *ctx, ibsn_ws_model *md, int64_t B, int64_t m, int64_t n, const float *fs,
            const float *fte, const float *fth)
{
    hipStream_t st = ctx_stream(ctx);
    const int64_t P = B * (m + n), T = B * n;
    for (int a : {A_X, A_H1, A_H2, A_E})
        WNEED(md->a32[a], P * (a == A_X ? NF : WID));
    for (int a : {A_X, A_H1, A_H2})
        WNEED(md->a16[a], P * (a == A_X ? NF : WID));
    WNEED(md->a32[A_XH], T * NFH);
    WNEED(md->a16[A_XH], T * NFH);
    WNEED(md->a32[A_OL], T);
    WNEED(md->a32[A_CTX], B * 2 * WID);
    WNEED(md->a16[A_CTX], B * 2 * WID);
    WNEED(md->a32[A_CB], B * WID);
    WNEED(md->a16[A_CB], B * WID);
    WNEED(md->a32[A_TMP], B * WID);
    for (int a : {A_Z1, A_Z2}) {
        WNEED(md->a32[a], T * WID);
        WNEED(md->a16[a], T * WID);
    }
    WNEED(md->a32[A_O], T);
    float *x32 = md->a32[A_X].p;
    WCK(hipMemcpyAsync(x32, fs, sizeof(float) * B * m * NF, hipMemcpyDeviceToDevice, st));
    WCK(hipMemcpyAsync(x32 + B * m * NF, fte, sizeof(float) * B * n * NF, hipMemcpyDeviceToDevice,
                       st));
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(P * NF)), dim3(256), 0, st, P * NF, (const float *)x32,
                       md->a16[A_X].p);
    WCK(hipMemcpyAsync(md->a32[A_XH].p, fth, sizeof(float) * T * NFH, hipMemcpyDeviceToDevice,
                       st));
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(T * NFH)), dim3(256), 0, st, T * NFH, fth,
                       md->a16[A_XH].p);
    const float *w = md->w.p;
    const bf16 *w16 = md->w16.p;
    const Param *p = md->prm;
    WCK(gemm(st, true, P, WID, NF, md->a16[A_X].p, NF, 1, w16 + p[P_W1].off, WID, 1,
             w + p[P_B1].off, nullptr, 1, md->a32[A_H1].p, md->a16[A_H1].p, WID));
    WCK(gemm(st, true, P, WID, WID, md->a16[A_H1].p, WID, 1, w16 + p[P_W2].off, WID, 1,
             w + p[P_B2].off, nullptr, 1, md->a32[A_H2].p, md->a16[A_H2].p, WID));
    WCK(gemm(st, false, P, WID, WID, md->a16[A_H2].p, WID, 1, w16 + p[P_W3].off, WID, 1,
             w + p[P_B3].off, nullptr, 1, md->a32[A_E].p, nullptr, WID));
    // mean pooling into CTX[b] = [h_s | h_t]
    float *ctxf = md->a32[A_CTX].p, *tmp = md->a32[A_TMP].p;
    for (int side = 0; side < 2; ++side) {
        const int64_t rows = side ? n : m;
        const float *src = md->a32[A_E].p + (side ? B * m * WID : 0);
        hipLaunchKernelGGL(k_group_sum, dim3(1, (unsigned)B), dim3(256), 0, st, (int)B, (int)rows,
                           WID, src, 1.0f / (float)rows, 0, tmp);
        WCK(hipMemcpy2DAsync(ctxf + side * WID, sizeof(float) * 2 * WID, tmp, sizeof(float) * WID,
                             sizeof(float) * WID, B, hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(B * 2 * WID)), dim3(256), 0, st, B * 2 * WID,
                       (const float *)ctxf, md->a16[A_CTX].p);
    // context c = CTX Wc + bc (B x 256); head z1 = relu(u Wf + bf), z2 = relu(z1 Wg + bg);
    // o_j = z2_j . c_b + bo, one product per instance
    WCK(gemm(st, false, B, WID, 2 * WID, md->a16[A_CTX].p, 2 * WID, 1, w16 + p[P_WC].off, WID, 1,
             w + p[P_BC].off, nullptr, 1, md->a32[A_CB].p, md->a16[A_CB].p, WID));
    WCK(gemm(st, true, T, WID, NFH, md->a16[A_XH].p, NFH, 1, w16 + p[P_WF].off, WID, 1,
             w + p[P_BF].off, nullptr, 1, md->a32[A_Z1].p, md->a16[A_Z1].p, WID));
    WCK(gemm(st, true, T, WID, WID, md->a16[A_Z1].p, WID, 1, w16 + p[P_WG].off, WID, 1,
             w + p[P_BG].off, nullptr, 1, md->a32[A_Z2].p, md->a16[A_Z2].p, WID));
    // linear path ol_j = ws . f_j (FP32), added to the readout as a per-row bias
    hipLaunchKernelGGL(k_lin_fwd, dim3(nblk(T)), dim3(256), 0, st, T,
                       (const float *)md->a32[A_XH].p, w + p[P_WS].off, md->a32[A_OL].p);
    for (int64_t b = 0; b < B; ++b)
        WCK(gemm(st, false, n, 1, WID, md->a16[A_Z2].p + b * n * WID, WID, 1,
                 md->a16[A_CB].p + b * WID, 1, 1, w + p[P_BO].off, md->a32[A_OL].p + b * n, 1,
                 md->a32[A_O].p + b * n, nullptr, 1));
    return IBSN_OK;
}

// relu backward of layer activation a: d32[a] *= (a32[a] > 0), BF16 copy in d16[a]
void relu_bwd(hipStream_t st, ibsn_ws_model *md, int a, int64_t cnt)
{
    hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(cnt)), dim3(256), 0, st, cnt, md->d32[a].p,
                       (const float *)md->a32[a].p, md->d16[a].p);
}

// Backward pass from dO = d32[A_O] (T values); writes every parameter's gradient into g.
int backward(ibsn_ctx *ctx, ibsn_ws_model *md, int64_t B, int64_t m, int64_t n)
{
    hipStream_t st = ctx_stream(ctx);
    const int64_t P = B * (m + n), T = B * n;
    for (int a : {A_H1, A_H2, A_E}) {
        WNEED(md->d32[a], P * WID);
        WNEED(md->d16[a], P * WID);
    }
    for (int a : {A_Z1, A_Z2}) {
        WNEED(md->d32[a], T * WID);
        WNEED(md->d16[a], T * WID);
    }
    WNEED(md->d16[A_O], T);
    WNEED(md->d32[A_CB], B * WID);
    WNEED(md->d16[A_CB], B * WID);
    WNEED(md->d32[A_CTX], B * 2 * WID);
    const Param *p = md->prm;
    float *g = md->g.p;
    const bf16 *w16 = md->w16.p;
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(T)), dim3(256), 0, st, T,
                       (const float *)md->d32[A_O].p, md->d16[A_O].p);
    // readout o_j = z2_j . c_b + ws . f_j + bo: dws = sum_j dO_j f_j, dz2_j = dO_j c_b,
    // dc_b = sum_j dO_j z2_j
    WCK(colsum(st, T, 1, md->d32[A_O].p, g + p[P_BO].off));
    hipLaunchKernelGGL(k_lin_grad, dim3(NFH), dim3(256), 0, st, T,
                       (const float *)md->a32[A_XH].p, (const float *)md->d32[A_O].p,
                       g + p[P_WS].off);
    for (int64_t b = 0; b < B; ++b) {
        WCK(gemm(st, false, n, WID, 1, md->d16[A_O].p + b * n, 1, 1, md->a16[A_CB].p + b * WID, 0,
                 1, nullptr, nullptr, 1, md->d32[A_Z2].p + b * n * WID, nullptr, WID));
        WCK(gemm(st, false, 1, WID, n, md->d16[A_O].p + b * n, 0, 1, md->a16[A_Z2].p + b * n * WID,
                 WID, 1, nullptr, nullptr, 1, md->d32[A_CB].p + b * WID, nullptr, WID));
    }
    relu_bwd(st, md, A_Z2, T * WID);
    // z2 = relu(z1 Wg + bg)
    WCK(gemm(st, false, WID, WID, T, md->a16[A_Z1].p, 1, WID, md->d16[A_Z2].p, WID, 1, nullptr,
             nullptr, 1, g + p[P_WG].off, nullptr, WID));
    WCK(colsum(st, T, WID, md->d32[A_Z2].p, g + p[P_BG].off));
    WCK(gemm(st, false, T, WID, WID, md->d16[A_Z2].p, WID, 1, w16 + p[P_WG].off, 1, WID, nullptr,
             nullptr, 1, md->d32[A_Z1].p, nullptr, WID));
    relu_bwd(st, md, A_Z1, T * WID);
    // z1 = relu(u Wf + bf)
    WCK(gemm(st, false, NFH, WID, T, md->a16[A_XH].p, 1, NFH, md->d16[A_Z1].p, WID, 1, nullptr,
             nullptr, 1, g + p[P_WF].off, nullptr, WID));
    WCK(colsum(st, T, WID, md->d32[A_Z1].p, g + p[P_BF].off));
    // c = CTX Wc + bc
    WCK(colsum(st, B, WID, md->d32[A_CB].p, g + p[P_BC].off));
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(B * WID)), dim3(256), 0, st, B * WID,
                       (const float *)md->d32[A_CB].p, md->d16[A_CB].p);
    WCK(gemm(st, false, 2 * WID, WID, B, md->a16[A_CTX].p, 1, 2 * WID, md->d16[A_CB].p, WID, 1,
             nullptr, nullptr, 1, g + p[P_WC].off, nullptr, WID));
    WCK(gemm(st, false, B, 2 * WID, WID, md->d16[A_CB].p, WID, 1, w16 + p[P_WC].off, 1, WID,
             nullptr, nullptr, 1, md->d32[A_CTX].p, nullptr, 2 * WID));
    // pooling: dE of the sources of b = dCTX[b][0:256] / m, of the targets dCTX[b][256:] / n
    hipLaunchKernelGGL(k_group_bcast, dim3(nblk(B * m * WID)), dim3(256), 0, st, B * m, (int)m,
                       WID, (const float *)md->d32[A_CTX].p, (int64_t)2 * WID, 1.0f / (float)m,
                       md->d32[A_E].p);
    hipLaunchKernelGGL(k_group_bcast, dim3(nblk(B * n * WID)), dim3(256), 0, st, B * n, (int)n,
                       WID, (const float *)(md->d32[A_CTX].p + WID), (int64_t)2 * WID,
                       1.0f / (float)n, md->d32[A_E].p + B * m * WID);
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(P * WID)), dim3(256), 0, st, P * WID,
                       (const float *)md->d32[A_E].p, md->d16[A_E].p);
    // e = h2 W3 + b3
    WCK(gemm(st, false, WID, WID, P, md->a16[A_H2].p, 1, WID, md->d16[A_E].p, WID, 1, nullptr,
             nullptr, 1, g + p[P_W3].off, nullptr, WID));
    WCK(colsum(st, P, WID, md->d32[A_E].p, g + p[P_B3].off));
    WCK(gemm(st, false, P, WID, WID, md->d16[A_E].p, WID, 1, w16 + p[P_W3].off, 1, WID, nullptr,
             nullptr, 1, md->d32[A_H2].p, nullptr, WID));
    relu_bwd(st, md, A_H2, P * WID);
    // h2 = relu(h1 W2 + b2)
    WCK(gemm(st, false, WID, WID, P, md->a16[A_H1].p, 1, WID, md->d16[A_H2].p, WID, 1, nullptr,
             nullptr, 1, g + p[P_W2].off, nullptr, WID));
    WCK(colsum(st, P, WID, md->d32[A_H2].p, g + p[P_B2].off));
    WCK(gemm(st, false, P, WID, WID, md->d16[A_H2].p, WID, 1, w16 + p[P_W2].off, 1, WID, nullptr,
             nullptr, 1, md->d32[A_H1].p, nullptr, WID));
    relu_bwd(st, md, A_H1, P * WID);
    // h1 = relu(x W1 + b1)
    WCK(gemm(st, false, NF, WID, P, md->a16[A_X].p, 1, NF, md->d16[A_H1].p, WID, 1, nullptr,
             nullptr, 1, g + p[P_W1].off, nullptr, WID));
    WCK(colsum(st, P, WID, md->d32[A_H1].p, g + p[P_B1].off));
    return IBSN_OK;
}

int check_dims(ibsn_ctx *ctx, int64_t B, int64_t m, int64_t n)
{
    if (B < 1 || m < 1 || n < 1 || B * (m + n) > (int64_t)1 << 28)
        return ctx_fail(ctx, IBSN_ERR_INVALID_ARG, "warm start: need B, m, n >= 1 and B (m+n) <= 2^28");
    return IBSN_OK;
}

}  // namespace

extern "C" {

int64_t ibsn_ws_param_count(void)
{
    Param p[NPARAM];
    return layout(p);
}

int ibsn_ws_create(ibsn_ctx *ctx, uint64_t seed, ibsn_ws_model **out)
{
    if (!ctx || !out)
        return IBSN_ERR_INVALID_ARG;
    *out = nullptr;
    WCK(hipSetDevice(ctx_device(ctx)));
    ibsn_ws_model *md = new ibsn_ws_model();
    md->ctx = ctx;
    md->total = layout(md->prm);
    const size_t N = (size_t)md->total;
    if (!md->w.ensure(N) || !md->g.ensure(N) || !md->m1.ensure(N) || !md->m2.ensure(N) ||
        !md->w16.ensure(N)) {
        ibsn_ws_free(md);
        return ctx_fail(ctx, IBSN_ERR_OOM, "warm-start parameters: out of memory");
    }
    // He initialisation of the matrices (normal, std sqrt(2 / inputs)); zero biases, a zero
    // linear path and a zero context map Wc, so that the output starts at 0 and the first
    // steps fit the linear path while the context grows from zero
    std::vector<float> h(N, 0.0f);
    std::mt19937_64 rng(seed);
    for (int i = 0; i < NPARAM; ++i) {
        const Param &p = md->prm[i];
        if (p.rows == 1 || i == P_WS || i == P_WC)
            continue;
        std::normal_distribution<float> nd(0.0f, sqrtf(2.0f / (float)p.rows));
        for (int64_t k = 0; k < (int64_t)p.rows * p.cols; ++k)
            h[p.off + k] = nd(rng);
    }
    const int rc = ibsn_ws_set_params(ctx, md, h.data(), md->total);
    if (rc != IBSN_OK) {
        ibsn_ws_free(md);
        return rc;
    }
    *out = md;
    return IBSN_OK;
}

void ibsn_ws_free(ibsn_ws_model *md)
{
    if (!md)
        return;
    md->w.release();
    md->g.release();
    md->m1.release();
    md->m2.release();
    md->part.release();
    md->w16.release();
    for (int a = 0; a < A_N; ++a) {
        md->a32[a].release();
        md->d32[a].release();
        md->a16[a].release();
        md->d16[a].release();
    }
    delete md;
}

int ibsn_ws_get_params(ibsn_ctx *ctx, const ibsn_ws_model *md, float *host, int64_t count)
{
    if (!ctx || !md || !host || count != md->total)
        return ctx ? ctx_fail(ctx, IBSN_ERR_INVALID_ARG, "get_params: count must be the parameter count")
                   : IBSN_ERR_INVALID_ARG;
    hipStream_t st = ctx_stream(ctx);
    WCK(hipMemcpyAsync(host, md->w.p, sizeof(float) * count, hipMemcpyDeviceToHost, st));
    WCK(hipStreamSynchronize(st));
    return IBSN_OK;
}

int ibsn_ws_set_params(ibsn_ctx *ctx, ibsn_ws_model *md, const float *host, int64_t count)
{
    if (!ctx || !md || !host || count != md->total)
        return ctx ? ctx_fail(ctx, IBSN_ERR_INVALID_ARG, "set_params: count must be the parameter count")
                   : IBSN_ERR_INVALID_ARG;
    hipStream_t st = ctx_stream(ctx);
    WCK(hipMemcpyAsync(md->w.p, host, sizeof(float) * count, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(count)), dim3(256), 0, st, count,
                       (const float *)md->w.p, md->w16.p);
    // fresh Adam state
    std::vector<float> z((size_t)count, 0.0f);
    WCK(hipMemcpyAsync(md->m1.p, z.data(), sizeof(float) * count, hipMemcpyHostToDevice, st));
    WCK(hipMemcpyAsync(md->m2.p, z.data(), sizeof(float) * count, hipMemcpyHostToDevice, st));
    WCK(hipStreamSynchronize(st));
    md->step = 0;
    return IBSN_OK;
}

int ibsn_ws_features(ibsn_ctx *ctx, const ibsn_problem *prob, const double *x, const double *y,
                     float *fs, float *fte, float *fth, double *scale_host)
{
    if (!ctx || !prob || !x || !y || !fs || !fte || !fth || !scale_host)
        return ctx ? ctx_fail(ctx, IBSN_ERR_INVALID_ARG, "ws_features: arguments required")
                   : IBSN_ERR_INVALID_ARG;
    const int64_t m = prob->m, n = prob->n;
    if (m < 1 || n < 1 || !prob->C || !prob->a || !prob->b)
        return ctx_fail(ctx, IBSN_ERR_INVALID_ARG, "ws_features: invalid problem");
    if (prob->cost_kind == IBSN_COST_POINTS && prob->ldc != 2)
        return ctx_fail(ctx, IBSN_ERR_INVALID_ARG, "ws_features: 2-D points only");
    WCK(hipSetDevice(ctx_device(ctx)));
    hipStream_t st = ctx_stream(ctx);
    // splits of the point list so that the potential kernel has about 2048 workgroups
    const int64_t tb = (n + 255) / 256, npts = m + n;
    int64_t splits = (2048 + tb - 1) / tb;
    splits = splits < 1 ? 1 : (splits > 64 ? 64 : splits);
    int64_t per = (npts + splits - 1) / splits;
    per = (per + 255) / 256 * 256;
    splits = (npts + per - 1) / per;
    double *buf = nullptr;
    const int64_t nbuf = PR_N + n + n * NGREEN + splits * n * NGREEN;
    WCK(hipMallocAsync((void **)&buf, sizeof(double) * nbuf, st));
    double *par = buf, *cm = buf + PR_N, *g = cm + n, *gpart = g + n * NGREEN;
    const bool pts = prob->cost_kind == IBSN_COST_POINTS;
    if (prob->cost_kind == IBSN_COST_F32)
        hipLaunchKernelGGL(k_box<float>, dim3(1), dim3(1024), 0, st, (int)m, (int)n, x, y,
                           (const float *)prob->C, prob->ldc, 0.0, par);
    else
        hipLaunchKernelGGL(k_box<double>, dim3(1), dim3(1024), 0, st, (int)m, (int)n, x, y,
                           pts ? nullptr : (const double *)prob->C, prob->ldc, prob->cost_scale,
                           par);
    if (prob->cost_kind == IBSN_COST_F64)
        hipLaunchKernelGGL(k_colmin<double>, dim3(nblk(n)), dim3(256), 0, st, (int)m, (int)n,
                           (const double *)prob->C, prob->ldc, cm);
    else if (prob->cost_kind == IBSN_COST_F32)
        hipLaunchKernelGGL(k_colmin<float>, dim3(nblk(n)), dim3(256), 0, st, (int)m, (int)n,
                           (const float *)prob->C, prob->ldc, cm);
    else
        hipLaunchKernelGGL(k_colmin_pts, dim3(nblk(n)), dim3(256), 0, st, (int)m, (int)n,
                           (int)prob->ldc, (const double *)prob->C, prob->y, prob->cost_scale, cm);
    hipLaunchKernelGGL(k_green, dim3((unsigned)tb, (unsigned)splits), dim3(256), 0, st, (int)m,
                       (int)n, (int)per, x, y, prob->a, prob->b, (const double *)par, gpart);
    hipLaunchKernelGGL(k_green_sum, dim3(nblk(n)), dim3(256), 0, st, (int)n, (int)splits,
                       (const double *)gpart, g);
    hipLaunchKernelGGL(k_feat_means, dim3(1), dim3(1024), 0, st, (int)n, (const double *)cm,
                       (const double *)g, par);
    hipLaunchKernelGGL(k_features, dim3(nblk(m > n ? m : n)), dim3(256), 0, st, (int)m, (int)n, x,
                       y, prob->a, prob->b, (const double *)cm, (const double *)g,
                       (const double *)par, fs, fte, fth);
    double ph[PR_N];
    WCK(hipMemcpyAsync(ph, par, sizeof(ph), hipMemcpyDeviceToHost, st));
    WCK(hipFreeAsync(buf, st));
    WCK(hipStreamSynchronize(st));
    *scale_host = ph[PR_U] * ph[PR_S];
    return IBSN_OK;
}

int ibsn_ws_forward(ibsn_ctx *ctx, ibsn_ws_model *md, int64_t B, int64_t m, int64_t n,
                    const float *fs, const float *fte, const float *fth, float *out)
{
    if (!ctx || !md || !fs || !fte || !fth || !out)
        return ctx ? ctx_fail(ctx, IBSN_ERR_INVALID_ARG, "ws_forward: arguments required")
                   : IBSN_ERR_INVALID_ARG;
    CKI(check_dims(ctx, B, m, n));
    WCK(hipSetDevice(ctx_device(ctx)));
    CKI(forward(ctx, md, B, m, n, fs, fte, fth));
    WCK(hipMemcpyAsync(out, md->a32[A_O].p, sizeof(float) * B * n, hipMemcpyDeviceToDevice,
                       ctx_stream(ctx)));
    return IBSN_OK;
}

int ibsn_ws_predict(ibsn_ctx *ctx, ibsn_ws_model *md, int64_t m, int64_t n, const float *fs,
                    const float *fte, const float *fth, double scale, double *gamma_out)
{
    if (!ctx || !md || !fs || !fte || !fth || !gamma_out || !(scale > 0.0))
        return ctx ? ctx_fail(ctx, IBSN_ERR_INVALID_ARG, "ws_predict: arguments required, scale > 0")
                   : IBSN_ERR_INVALID_ARG;
    CKI(check_dims(ctx, 1, m, n));
    WCK(hipSetDevice(ctx_device(ctx)));
    CKI(forward(ctx, md, 1, m, n, fs, fte, fth));
    hipLaunchKernelGGL(k_predict_out, dim3(1), dim3(256), 0, ctx_stream(ctx), (int)n,
                       (const float *)md->a32[A_O].p, scale, gamma_out);
    WCK(hipGetLastError());
    return IBSN_OK;
}

int ibsn_ws_train_step(ibsn_ctx *ctx, ibsn_ws_model *md, int64_t B, int64_t m, int64_t n,
                       const float *fs, const float *fte, const float *fth, const float *target,
                       float lr, float *loss_host, float *grad_host)
{
    if (!ctx || !md || !fs || !fte || !fth || !target || !loss_host || !(lr >= 0.0f))
        return ctx ? ctx_fail(ctx, IBSN_ERR_INVALID_ARG, "ws_train_step: arguments required")
                   : IBSN_ERR_INVALID_ARG;
    CKI(check_dims(ctx, B, m, n));
    WCK(hipSetDevice(ctx_device(ctx)));
    hipStream_t st = ctx_stream(ctx);
    CKI(forward(ctx, md, B, m, n, fs, fte, fth));
    const int64_t T = B * n;
    WNEED(md->d32[A_O], T);
    WNEED(md->part, B);
    hipLaunchKernelGGL(k_head_loss, dim3((unsigned)B), dim3(256), 0, st, (int)n,
                       (const float *)md->a32[A_O].p, target, 1.0f / (float)T, md->part.p,
                       md->d32[A_O].p);
    CKI(backward(ctx, md, B, m, n));
    if (grad_host)
        WCK(hipMemcpyAsync(grad_host, md->g.p, sizeof(float) * md->total, hipMemcpyDeviceToHost,
                           st));
    std::vector<float> part((size_t)B);
    WCK(hipMemcpyAsync(part.data(), md->part.p, sizeof(float) * B, hipMemcpyDeviceToHost, st));
    if (lr > 0.0f) {
        ++md->step;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - powf(b1, (float)md->step), c2 = 1.0f - powf(b2, (float)md->step);
        hipLaunchKernelGGL(k_adam, dim3(nblk(md->total)), dim3(256), 0, st, md->total, md->w.p,
                           (const float *)md->g.p, md->m1.p, md->m2.p, md->w16.p, lr, b1, b2,
                           1e-8f, c1, c2);
        WCK(hipGetLastError());
    }
    WCK(hipStreamSynchronize(st));
    double l = 0.0;
    for (float v : part)
        l += v;
    *loss_host = (float)(l / (double)T);
    return IBSN_OK;
}

}  // extern "C"
