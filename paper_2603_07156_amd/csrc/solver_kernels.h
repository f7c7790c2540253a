// solver_kernels.h -- device scalar slots and launchers of solver_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibsn {

// slots of the device scalar array (doubles)
enum {
    SC_GN2 = 0, SC_GN, SC_G1,               // ||g||^2, ||g||, ||g||_1
    SC_BIG, SC_TAUSHIFT,                    // Armijo trial form
    SC_OBJ, SC_DL, SC_GD, SC_BD, SC_ROWSUM, // objective, dL, g^T Delta, b^T Delta, part sum
    SC_BG, SC_BP, SC_ER1, SC_COLRES,        // stop test
    SC_SUMA, SC_SUMB, SC_MINA, SC_MINB, SC_BAD, SC_ISTAR,
    SC_NNZ,                                 // (as double) nnz of the last factor
    SC_WMAX, SC_CMAX, SC_TB,                // max|s+gamma/eta|, max|C|, b^T tau
    SC_BB,                                  // b^T b (mixed-precision switch, Delta_kkt)
    SC_AA,                                  // a^T a (Delta_kkt)
    SC_CMIN,                                // min_j c_j (Sinkhorn: log-domain step below ~1e-290)
    SC_NSLOT = 32
};

hipError_t sk_gnorms(int64_t n, const double *g, double *scal, hipStream_t st);
// Sinkhorn step on the two-level potential (w, wlo) from lc = log c (split = 0: steps on the
// grid); (w, wlo) += d; lc = log c
hipError_t sk_sinkhorn_step(int64_t n, double eta, double q, int split, const double *b,
                            const double *lc, const double *s, double *w, double *wlo,
                            hipStream_t st);
hipError_t sk_dd_axpy(int64_t n, double q, const double *d, double *w, double *wlo, hipStream_t st);
hipError_t sk_log(int64_t n, const double *c, double *lc, hipStream_t st);
hipError_t sk_wmax(int64_t n, const double *s, const double *gamma, double eta, double *scal,
                   hipStream_t st);
// scal[SC_CMAX] = max |C| (part: G doubles of scratch)
hipError_t sk_cost_max(int64_t m, int64_t n, int64_t ldc, int kind, const void *C,
                       const double *py, double pscale, double *part, int G, double *scal,
                       hipStream_t st);
hipError_t sk_gamma_of(int64_t n, double eta, const double *w, const double *wlo, const double *s,
                       double *gamma, hipStream_t st);
hipError_t sk_center(int64_t n, double *gamma, hipStream_t st);
hipError_t sk_trial_prep(int64_t n, double t, double eta, double q, int split, const double *Delta,
                         const double *b, double *tau, double *colv, double *scal, hipStream_t st);
// scal[slot] = alpha * (op-reduce_g part[g*stride+off]) + beta * scal[src] (src < 0: none);
// op 0 = sum, 1 = max, 2 = min
hipError_t sk_sum_parts(int G, int stride, int off, const double *part, double alpha, double beta,
                        int src, int slot, int op, double *scal, hipStream_t st);
hipError_t sk_dot_slot(int64_t n, const double *x, const double *y, int slot, double *scal,
                       hipStream_t st);
hipError_t sk_stop_prep(int64_t n, double sigma, const double *b, const double *w,
                        const double *wlo, const double *gamma, const double *colX,
                        const double *colF, double *y, double *ec, double *psi, double *scal,
                        hipStream_t st);
// x[0..n) = v (a kernel: safe under graph capture)
hipError_t sk_fill(int64_t n, double v, double *x, hipStream_t st);
// certificate and Delta_kkt from the stop passes' partials; needs scal[SC_AA], scal[SC_BB]
hipError_t sk_stop_final(int G, const double *part, const double *rowres_part, int G1,
                         double *scal, double *out, hipStream_t st);
hipError_t sk_problem_scalars(int64_t m, int64_t n, const double *a, const double *b,
                              double *scal, int *istar, hipStream_t st);
hipError_t sk_outer_update(int64_t m, int64_t n, const double *a, const double *M, const double *S,
                           const double *w, const double *wlo, double *r, double *s, hipStream_t st);
hipError_t sk_init_center(int64_t m, int64_t n, const double *a, const double *b, double *r,
                          double *s, hipStream_t st);
hipError_t sk_axpy(int64_t n, double alpha, const double *x, double *y, hipStream_t st);
hipError_t sk_neg(int64_t n, const double *x, double *y, hipStream_t st);
hipError_t sk_zero_i32(int64_t count, int32_t *x, hipStream_t st);

}  // namespace ibsn
