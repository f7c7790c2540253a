/*
 * ibsn_oracle.c -- plain FP64 CPU reference of the Inexact Bregman Sparse Newton
 * (IBSN) method for exact optimal transport.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * do.  It shares no code, header, table or helper with the HIP implementation.
 *
 * Problem (eq. (1)): min <C,X> over X>=0 with X1=a, X^T1=b.
 * Outer loop (eq. (3), Algorithm 2): X^{k+1} ~ argmin <C,X> + eta*D_phi(X,X^k).
 * Semi-dual subproblem (eq. (6)):
 *     L^k(gamma) = -b^T gamma + eta * sum_i a_i log sum_j X^k_ij exp((gamma_j-C_ij)/eta).
 *
 * Prox centre held implicitly.  X^0 = a b^T (Algorithm 2 input) and
 * X^{k+1} = diag(a) P^k(gamma) (eq. (7)) give, for every k,
 *     log X^k_ij = r_i + s_j - k*C_ij/eta,
 * with r = log a, s = log b at k = 0 and r <- log a - lse(gamma), s <- s + gamma/eta
 * at each outer update.  The row constant r_i cancels in P (eq. (7)), so the plan of
 * the subproblem at gamma is a row softmax of
 *     theta_ij = w_j - sigma*C_ij,   sigma = (k+1)/eta,   w_j = s_j + gamma_j/eta,
 * and the row log-normaliser of eq. (5) is r_i + lse_i with lse_i = LSE_j theta_ij.
 *
 * Exact exponents.  w_j and theta_ij grow like sigma, but P only needs the small
 * differences theta_ij - (row shift).  Both the column potentials w_j and the row
 * shifts M_i are kept on a grid of spacing q (a power of two, 2^(e-50) for a bound
 * 2^(e-1) <= |w|, |theta| < 2^e), so w_j - M_i is an exact double and
 *     x_ij = fma(-sigma, C_ij, w_j - M_i) = theta_ij - M_i
 * carries one rounding at the scale of x_ij itself (|x| <= ~40 for every entry that
 * matters) instead of one at the scale of sigma.  Rounding a value v to the grid is
 * grid(v) = q * rint(v / q) (exact operations for a power-of-two q).
 *
 * Two sets of passes.  The grid passes (orc_eval, orc_trial, orc_sparsify, orc_stop) follow
 * the solver's exact-exponent scheme described here and drive orc_solve.  The plain passes
 * at the end of the file (orc_plain_eval, orc_plain_sparsify, orc_plain_stop) take the same
 * quantities straight from their definitions, with no grid; they are the reference that the
 * grid scheme (here and in any other implementation) is held to, within the bound that the
 * grid's rounding of w sets.
 *
 * Row state.  A pair (M_i, S_i), M_i on the grid, represents
 *     P_ij = exp(x_ij) / S_i,   x_ij = fma(-sigma, C_ij, w_j - M_i),
 * which is eq. (7) with the common factor exp(-M_i) cancelled.  A fresh evaluation
 * sets M_i = grid(max_j theta_ij) and S_i = sum_j exp(x_ij).
 *
 * Conventions fixed where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *  - i* = lowest index among the maxima of a (Algorithm 1 input).
 *  - threshold test P_ij >= rho is inclusive (Algorithm 1, step 3).
 *  - norms of g in rho and in the shift are Euclidean (notation paragraph).
 *  - CG starts from 0 and stops when ||r|| <= max(min(0.1, ||g||), cg_rtol_min)*||g||
 *    or at cg_maxit.
 *  - Armijo decrease L(gamma+t*Delta)-L(gamma) is evaluated in difference form on the
 *    grid-rounded step, see orc_trial(); only a finite decrease is accepted.
 *  - Sinkhorn warm-up re-centres gamma after every gamma-step (centering does not
 *    change P, g or the Newton iterates: L(gamma + c1) = L(gamma) since 1^T b = 1 = 1^T a).
 *  - the inner loop also ends when the gradient gate has passed but the D_phi test has
 *    failed stall_limit times in the same outer iteration (the test has a rounding floor).
 *  - Column sums are accumulated over 64 fixed row chunks, in chunk order, so results
 *    do not depend on the number of OpenMP threads.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NCHUNK 64

/* status codes */
#define ORC_OK 0
#define ORC_WARN_MAXITER 1
#define ORC_ERR_ARG (-1)
#define ORC_ERR_NUMERIC (-4)

/* cost element: kind 0 = float64, kind 1 = float32 (widened exactly to double) */
static inline double cost_at(const void *C, int kind, int64_t ldc, int64_t i, int64_t j)
{
    if (kind == 1)
        return (double)((const float *)C)[i * ldc + j];
    return ((const double *)C)[i * ldc + j];
}

/* round v to the grid of spacing q (q a power of two) */
static inline double grid(double v, double q) { return q * rint(v / q); }

/* x_ij = theta_ij - M_i for the potential w_j + wl_j (wl may be NULL: 0), with w_j - M_i
   exact (both on the grid) */
static inline double xval(const void *C, int kind, int64_t ldc, int64_t i, int64_t j,
                          double sigma, const double *w, const double *wl, double Mi)
{
    double x = fma(-sigma, cost_at(C, kind, ldc, i, j), w[j] - Mi);
    return wl ? x + wl[j] : x;
}

/* Knuth's two-sum: hi + lo = a + b exactly, hi = fl(a + b) */
static inline void two_sum(double a, double b, double *hi, double *lo)
{
    double h = a + b;
    double bv = h - a;
    double av = h - bv;
    *hi = h;
    *lo = (a - av) + (b - bv);
}

/* (w, wl) += d with w kept on the grid of spacing q: the exact sum wl + d is split into
   its grid part (added to w, exactly) and the remainder */
static inline void pot_add(double *w, double *wl, double d, double q)
{
    double u, e;
    two_sum(*wl, d, &u, &e);
    double gpart = grid(u, q);
    *w += gpart;
    *wl = (u - gpart) + e;
}

static double dot(int64_t n, const double *x, const double *y)
{
    double acc = 0.0;
    for (int64_t j = 0; j < n; ++j)
        acc += x[j] * y[j];
    return acc;
}

static double nrm2(int64_t n, const double *x) { return sqrt(dot(n, x, x)); }

/* grid spacing for values bounded by B: 2^(e-50) with 2^(e-1) <= B < 2^e; values up to
   2^(e+1) in magnitude are then multiples of q and differences of two of them are exact */
double orc_quantum(double B)
{
    if (!(B >= 1.0))
        B = 1.0;
    return ldexp(1.0, ilogb(B) + 1 - 50);
}

double orc_cost_max(int64_t m, int64_t n, const void *C, int kind, int64_t ldc)
{
    double mx = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double c = fabs(cost_at(C, kind, ldc, i, j));
            if (c > mx)
                mx = c;
        }
    return mx;
}

/* quantum of an outer iteration: bound max_j |s_j + gamma_j/eta| + sigma * max|C| */
double orc_center_quantum(int64_t n, const double *s, const double *gamma, double eta,
                          int64_t k, double cmax)
{
    double mw = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double v = fabs(s[j] + gamma[j] / eta);
        if (v > mw)
            mw = v;
    }
    return orc_quantum(mw + ((double)(k + 1) / eta) * cmax);
}

/* Two-level potentials w_j + wl_j = s_j + gamma_j / eta: w_j = grid(s_j + gamma_j / eta)
   and wl_j the remainder, carried exactly up to one rounding at its own size (the rounding
   of s_j + d_j from a two-sum, that of d_j = gamma_j / eta from its fma residual).
   wl == NULL: the potentials are kept on the grid (w_j only). */
void orc_make_w(int64_t n, const double *s, const double *gamma, double eta, double q, double *w,
                double *wl)
{
    for (int64_t j = 0; j < n; ++j) {
        double d = gamma[j] / eta;
        double t, e;
        two_sum(s[j], d, &t, &e);
        w[j] = grid(t, q);
        if (wl) {
            double rd = fma(-d, eta, gamma[j]); /* gamma_j - d eta, exactly */
            wl[j] = ((t - w[j]) + e) + rd / eta;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Eval pass: eq. (5) (best zeta as a row LSE), eq. (6) (objective), eq. (7) (P)  */
/* and eq. (8) (gradient g = P^T a - b), at the grid potentials w.                 */
/* The objective uses the gamma given (gamma = eta (w - s) up to the grid).         */
/* ------------------------------------------------------------------------- */
int orc_eval(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, int64_t k, double eta,
             double q, const double *w, const double *wl, const double *r, const double *gamma,
             const double *a,
             const double *b, double *M, double *S, double *c, double *g, double *L,
             double *plan /* m*n (row-major) or NULL */)
{
    if (m < 1 || n < 1 || !(eta > 0) || !(q > 0))
        return ORC_ERR_ARG;
    const double sigma = (double)(k + 1) / eta;

    /* row shift (grid-rounded maximum) and row sum of exp(theta - shift) */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double mx = -INFINITY;
        for (int64_t j = 0; j < n; ++j) {
            double th = fma(-sigma, cost_at(C, kind, ldc, i, j), w[j]);
            if (th > mx)
                mx = th;
        }
        double Mi = grid(mx, q);
        double sum = 0.0;
        for (int64_t j = 0; j < n; ++j)
            sum += exp(xval(C, kind, ldc, i, j, sigma, w, wl, Mi));
        M[i] = Mi;
        S[i] = sum;
    }

    /* column marginals c_j = sum_i a_i P_ij */
    double *part = calloc((size_t)ORC_NCHUNK * n, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int q = 0; q < ORC_NCHUNK; ++q) {
        int64_t i0 = m * q / ORC_NCHUNK, i1 = m * (q + 1) / ORC_NCHUNK;
        double *pc = part + (size_t)q * n;
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t j = 0; j < n; ++j) {
                double p = exp(xval(C, kind, ldc, i, j, sigma, w, wl, M[i])) / S[i];
                pc[j] += a[i] * p;
                if (plan)
                    plan[i * n + j] = a[i] * p;
            }
    }
    for (int64_t j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int q = 0; q < ORC_NCHUNK; ++q)
            acc += part[(size_t)q * n + j];
        c[j] = acc;
        g[j] = acc - b[j];
    }
    free(part);

    /* L = -b^T gamma + eta * sum_i a_i (r_i + M_i + log S_i) */
    if (L && r && gamma) {
        double t = 0.0;
        for (int64_t i = 0; i < m; ++i)
            t += a[i] * (r[i] + M[i] + log(S[i]));
        *L = -dot(n, b, gamma) + eta * t;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Armijo trial (Algorithm 2, step 9) from the row state M of the point w.          */
/* The step is tau_j = t * Delta_j / eta (rounded to the grid when the potentials    */
/* are kept on it); the trial point is w + tau.  Exact algebra for the change:      */
/*   L(w + tau) - L(w) = -eta * b^T tau + eta * sum_i a_i delta_i,                  */
/*   delta_i = log( sum_j q_ij e^{tau_j} / sum_j q_ij ),  q_ij = exp(x_ij).           */
/* Small steps (max tau <= 500): delta_i = log1p(B_i / A_i) with A_i = sum_j q_ij,  */
/* B_i = sum_j q_ij expm1(tau_j), which keeps full relative precision when tau is   */
/* tiny; otherwise delta_i = tau_max + log(Z_i / A_i) with the shifted factors      */
/* exp(tau_j - tau_max).  The trial plan is P'_ij = qe_ij / Z_i with                */
/* qe_ij = q_ij e^{tau_j - shift}, Z_i = sum_j qe_ij; its column sums give c', g'.  */
/* New row state: M'_i = grid(M_i + shift + log max_j qe_ij) and                     */
/* S'_i = Z_i exp((M_i - M'_i) + shift), so exp(x'_ij)/S'_i = P'_ij for the fresh    */
/* x' of the point w + tau.  A row whose factors all underflow gives delta = +inf.  */
/* ------------------------------------------------------------------------- */
int orc_trial(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, int64_t k, double eta,
              double q, const double *w, const double *wl, const double *a, const double *b,
              const double *M,
              const double *Delta, double t, double *dL /* out */, double *tau_out /* n or NULL */,
              double *M_new, double *S_new, double *c_new, double *g_new)
{
    if (m < 1 || n < 1 || !(eta > 0) || !(q > 0))
        return ORC_ERR_ARG;
    const double sigma = (double)(k + 1) / eta;
    double *tau = malloc(sizeof(double) * n);
    double *cv = malloc(sizeof(double) * n);
    double *delta = malloc(sizeof(double) * m);
    double *Z = malloc(sizeof(double) * m);
    double tau_max = -INFINITY;
    for (int64_t j = 0; j < n; ++j) {
        /* with two-level potentials the step is taken as it is; on the grid otherwise */
        tau[j] = wl ? t * Delta[j] / eta : grid(t * Delta[j] / eta, q);
        if (tau[j] > tau_max)
            tau_max = tau[j];
    }
    const int small_step = tau_max <= 500.0;
    const double shift = small_step ? 0.0 : tau_max;
    for (int64_t j = 0; j < n; ++j)
        cv[j] = small_step ? expm1(tau[j]) : exp(tau[j] - tau_max);

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double A = 0.0, B = 0.0, Zi = 0.0, qmax = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double qv = exp(xval(C, kind, ldc, i, j, sigma, w, wl, M[i]));
            A += qv;
            double qe;
            if (small_step) {
                double qf = qv * cv[j];
                B += qf;
                qe = qv + qf;
            } else {
                qe = qv * cv[j];
            }
            Zi += qe;
            if (qe > qmax)
                qmax = qe;
        }
        if (!(Zi > 0.0)) {
            delta[i] = INFINITY;
            M_new[i] = M[i];
            S_new[i] = NAN;
        } else {
            delta[i] = small_step ? log1p(B / A) : shift + log(Zi / A);
            double Mn = grid(M[i] + (shift + log(qmax)), q);
            M_new[i] = Mn;
            S_new[i] = Zi * exp((M[i] - Mn) + shift);
        }
        Z[i] = Zi;
    }

    double *part = calloc((size_t)ORC_NCHUNK * n, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int qq = 0; qq < ORC_NCHUNK; ++qq) {
        int64_t i0 = m * qq / ORC_NCHUNK, i1 = m * (qq + 1) / ORC_NCHUNK;
        double *pc = part + (size_t)qq * n;
        for (int64_t i = i0; i < i1; ++i) {
            if (!(Z[i] > 0.0))
                continue;
            for (int64_t j = 0; j < n; ++j) {
                double qv = exp(xval(C, kind, ldc, i, j, sigma, w, wl, M[i]));
                double qe = small_step ? qv + qv * cv[j] : qv * cv[j];
                pc[j] += a[i] * (qe / Z[i]);
            }
        }
    }
    for (int64_t j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int qq = 0; qq < ORC_NCHUNK; ++qq)
            acc += part[(size_t)qq * n + j];
        c_new[j] = acc;
        g_new[j] = acc - b[j];
    }
    free(part);

    double sd = 0.0;
    for (int64_t i = 0; i < m; ++i)
        sd += a[i] * delta[i];
    *dL = -eta * dot(n, b, tau) + eta * sd;
    if (tau_out)
        memcpy(tau_out, tau, sizeof(double) * n);
    free(tau); free(cv); free(delta); free(Z);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1: Hessian sparsification.  P_ij = exp(x_ij)/S_i.                      */
/* For i != i*: keep P_ij >= rho and divide the kept entries by their sum.          */
/* Row i* is copied whole.  Output CSR (row_ptr[m+1], col[nnz], val[nnz]) in row    */
/* order, columns ascending, and d = P_rho^T a.                                     */
/* Returns nnz, or -(needed nnz) - 1 when cap is too small (nothing else written    */
/* except row_ptr).  A row whose entries all fall below rho is left empty.          */
/* ------------------------------------------------------------------------- */
int64_t orc_sparsify(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, int64_t k,
                     double eta, const double *w, const double *wl, const double *a, const double *M,
                     const double *S, double rho, int64_t istar, int64_t cap, int64_t *row_ptr,
                     int32_t *col, double *val, double *d)
{
    const double sigma = (double)(k + 1) / eta;
    int64_t *cnt = malloc(sizeof(int64_t) * m);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        if (i == istar) {
            cnt[i] = n;
            continue;
        }
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            double p = exp(xval(C, kind, ldc, i, j, sigma, w, wl, M[i])) / S[i];
            if (p >= rho)
                ++c;
        }
        cnt[i] = c;
    }
    row_ptr[0] = 0;
    for (int64_t i = 0; i < m; ++i)
        row_ptr[i + 1] = row_ptr[i] + cnt[i];
    int64_t nnz = row_ptr[m];
    free(cnt);
    if (nnz > cap)
        return -nnz - 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        int64_t o = row_ptr[i];
        double kappa = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double p = exp(xval(C, kind, ldc, i, j, sigma, w, wl, M[i])) / S[i];
            if (i == istar || p >= rho) {
                col[o] = (int32_t)j;
                val[o] = p;
                kappa += p;
                ++o;
            }
        }
        if (i != istar && kappa > 0.0)
            for (int64_t e = row_ptr[i]; e < o; ++e)
                val[e] = val[e] / kappa;
    }
    /* d = P_rho^T a (serial scatter in row order) */
    for (int64_t j = 0; j < n; ++j)
        d[j] = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            d[col[e]] += a[i] * val[e];
    return nnz;
}

/* H_rho v = (diag(P_rho^T a) v - P_rho^T diag(a) P_rho v)/eta  (Algorithm 1, step 4),
   plus shift*v (Algorithm 2, step 8).  H_rho is never formed. */
void orc_hvp(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
             const double *d, const double *a, double eta, double shift, const double *v,
             double *y)
{
    double *u = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *wv = calloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double acc = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            acc += val[e] * v[col[e]];
        u[i] = acc;
    }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            wv[col[e]] += val[e] * (a[i] * u[i]);
    for (int64_t j = 0; j < n; ++j)
        y[j] = (d[j] * v[j] - wv[j]) / eta + shift * v[j];
    free(u);
    free(wv);
}

/* Conjugate gradients for (H_rho + shift I) x = rhs, x0 = 0 (Algorithm 2, step 8;
   CG on the complement of the kernel span{1}, Theorem 3.2 and the text after it).
   Stops when ||r|| <= tol or after maxit iterations.  Returns the iteration count. */
int orc_cg(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
           const double *d, const double *a, double eta, double shift, const double *rhs,
           double tol, int maxit, double *x)
{
    double *r = malloc(sizeof(double) * n), *p = malloc(sizeof(double) * n),
           *Ap = malloc(sizeof(double) * n);
    for (int64_t j = 0; j < n; ++j) {
        x[j] = 0.0;
        r[j] = rhs[j];
        p[j] = rhs[j];
    }
    double rr = dot(n, r, r);
    int it = 0;
    while (sqrt(rr) > tol && it < maxit) {
        orc_hvp(m, n, row_ptr, col, val, d, a, eta, shift, p, Ap);
        double pAp = dot(n, p, Ap);
        if (!(pAp > 0.0))
            break;
        double alpha = rr / pAp;
        for (int64_t j = 0; j < n; ++j) {
            x[j] += alpha * p[j];
            r[j] -= alpha * Ap[j];
        }
        double rr_new = dot(n, r, r);
        double beta = rr_new / rr;
        for (int64_t j = 0; j < n; ++j)
            p[j] = r[j] + beta * p[j];
        rr = rr_new;
        ++it;
    }
    free(r); free(p); free(Ap);
    return it;
}

/* ------------------------------------------------------------------------- */
/* Inexact stop test and certificate.                                              */
/* X_ij = a_i P_ij with P from the row state.  Algorithm 3 (rounding onto Omega,    */
/* literal: y uses the column sums of X), then                                      */
/*   D_phi(Xhat, X) = sum Xhat log(Xhat/X) - Xhat + X          (eq. (3)),           */
/* evaluated with log X_ij = log a_i + x_ij - log S_i so that an X that underflows   */
/* does not make the term infinite; 0 log 0 = 0.                                     */
/* Certificate: for a dual vector v, zeta_i = min_j (C_ij - v_j) (c-transform,       */
/* appendix C.1) makes (zeta, v) feasible for the dual LP, so a^T zeta + b^T v is a  */
/* lower bound on the optimum; <C,Xhat> is an upper bound.  Two vectors are tried:   */
/* gamma itself (the paper's choice) and the entropic potential of the current plan, */
/* psi_j = (w_j - log b_j)/sigma (X_ij = a_i b_j exp(sigma (f_i + psi_j - C_ij))),    */
/* and the larger bound is reported.  The relative KKT residual of appendix C.1 is   */
/* evaluated for (X, gamma, zeta^c(gamma)).                                          */
/* out[0] = D_phi, out[1] = <C,Xhat>, out[2] = best dual bound, out[3] = <C,X>,     */
/* out[4] = Delta_kkt, out[5] = min Xhat, out[6] = ||e_r||_1, out[7] = <X,U>,        */
/* out[8] = dual bound from gamma, out[9] = dual bound from psi.                      */
/* ------------------------------------------------------------------------- */
/* Algorithm 3, steps 2-10, for a nonnegative X (m*n): z_i = min(a_i / sum_j X_ij, 1),
   y_j = min(b_j / sum_i X_ij, 1) (the column sums of X itself, as the algorithm states),
   F = diag(z) X diag(y), e_r = a - F 1, e_c = b - F^T 1.  colX (n) receives X^T 1.
   Returns ||e_r||_1. */
static double alg3_factors(int64_t m, int64_t n, const double *X, const double *a,
                           const double *b, double *z, double *y, double *er, double *ec,
                           double *colX)
{
    double *colF = calloc((size_t)n, sizeof(double));
    for (int64_t i = 0; i < m; ++i) {
        double rs = 0.0;
        for (int64_t j = 0; j < n; ++j)
            rs += X[i * n + j];
        z[i] = fmin(a[i] / rs, 1.0);
    }
    for (int64_t j = 0; j < n; ++j)
        colX[j] = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            colX[j] += X[i * n + j];
    for (int64_t j = 0; j < n; ++j)
        y[j] = fmin(b[j] / colX[j], 1.0);
    double er1 = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double rs = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double f = z[i] * X[i * n + j] * y[j];
            rs += f;
            colF[j] += f;
        }
        /* z <= 1 and y <= 1 make e_r, e_c >= 0 exactly; a negative value is rounding */
        er[i] = fmax(a[i] - rs, 0.0);
        er1 += er[i];
    }
    for (int64_t j = 0; j < n; ++j)
        ec[j] = fmax(b[j] - colF[j], 0.0);
    free(colF);
    return er1;
}

/* Algorithm 3 on a nonnegative X (m*n): the feasible plan xhat = F + e_r e_c^T / ||e_r||_1
   (F when ||e_r||_1 = 0).  z, y, er, ec (optional) receive the algorithm's vectors. */
void orc_round(int64_t m, int64_t n, const double *X, const double *a, const double *b,
               double *xhat, double *z_out, double *y_out, double *er_out, double *ec_out)
{
    double *z = malloc(sizeof(double) * m), *er = malloc(sizeof(double) * m);
    double *y = malloc(sizeof(double) * n), *ec = malloc(sizeof(double) * n);
    double *colX = malloc(sizeof(double) * n);
    const double er1 = alg3_factors(m, n, X, a, b, z, y, er, ec, colX);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            const double f = z[i] * X[i * n + j] * y[j];
            xhat[i * n + j] = er1 > 0.0 ? f + er[i] * ec[j] / er1 : f;
        }
    if (z_out)
        memcpy(z_out, z, sizeof(double) * m);
    if (y_out)
        memcpy(y_out, y, sizeof(double) * n);
    if (er_out)
        memcpy(er_out, er, sizeof(double) * m);
    if (ec_out)
        memcpy(ec_out, ec, sizeof(double) * n);
    free(z); free(er); free(y); free(ec); free(colX);
}

/* Algorithm 3 and the certificate for a plan given entry by entry: X (m*n) and its
   logarithm logX (m*n, finite where X underflows), the dual vectors gamma and psi (n).
   Optional outputs: xhat (m*n), and Algorithm 3's z (m), y (n), e_r (m), e_c (n). */
static void stop_from_plan(int64_t m, int64_t n, const void *C, int kind, int64_t ldc,
                           const double *X, const double *logX, const double *gamma,
                           const double *psi, const double *a, const double *b, double *out,
                           double *xhat, double *z_out, double *y_out, double *er_out,
                           double *ec_out)
{
    double *z = malloc(sizeof(double) * m), *er = malloc(sizeof(double) * m);
    double *colX = malloc(sizeof(double) * n);
    double *y = malloc(sizeof(double) * n), *ec = malloc(sizeof(double) * n);
    double *zc = malloc(sizeof(double) * m);
    /* Algorithm 3, steps 2-10 */
    const double er1 = alg3_factors(m, n, X, a, b, z, y, er, ec, colX);

    /* step 11 and the divergence / certificate sums (each row summed on its own, then the
       row totals: a single running sum over m*n terms loses accuracy at large m*n) */
    double dphi = 0.0, cxh = 0.0, cx = 0.0, xmin = INFINITY, xu = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double r_dphi = 0.0, r_cxh = 0.0, r_cx = 0.0, r_xu = 0.0;
        double zmin = INFINITY;
        for (int64_t j = 0; j < n; ++j) {
            double u = cost_at(C, kind, ldc, i, j) - gamma[j];
            if (u < zmin)
                zmin = u;
        }
        zc[i] = zmin;
        for (int64_t j = 0; j < n; ++j) {
            double x = X[i * n + j];
            double f = z[i] * x * y[j];
            double xh = er1 > 0.0 ? f + er[i] * ec[j] / er1 : f;
            double cij = cost_at(C, kind, ldc, i, j);
            if (xhat)
                xhat[i * n + j] = xh;
            if (xh > 0.0)
                r_dphi += xh * (log(xh) - logX[i * n + j]) - xh + x;
            else
                r_dphi += x;
            r_cxh += cij * xh;
            r_cx += cij * x;
            if (xh < xmin)
                xmin = xh;
            r_xu += x * ((cij - gamma[j]) - zmin);
        }
        dphi += r_dphi;
        cxh += r_cxh;
        cx += r_cx;
        xu += r_xu;
    }
    double dual_g = dot(m, a, zc) + dot(n, b, gamma);
    double dual_p = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double zmin = INFINITY;
        for (int64_t j = 0; j < n; ++j) {
            double u = cost_at(C, kind, ldc, i, j) - psi[j];
            if (u < zmin)
                zmin = u;
        }
        dual_p += a[i] * zmin;
    }
    dual_p += dot(n, b, psi);
    double dual = fmax(dual_g, dual_p);

    /* Delta_kkt (appendix C.1) for (X, gamma, zeta^c); U >= 0 by construction */
    double rr = 0.0, cc = 0.0, xf = 0.0, cf = 0.0, neg = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double rs = 0.0, r_xf = 0.0, r_neg = 0.0, r_cf = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double x = X[i * n + j];
            rs += x;
            r_xf += x * x;
            if (x < 0.0)
                r_neg += x * x;
            double cij = cost_at(C, kind, ldc, i, j);
            r_cf += cij * cij;
        }
        xf += r_xf;
        neg += r_neg;
        cf += r_cf;
        rr += (rs - a[i]) * (rs - a[i]);
    }
    for (int64_t j = 0; j < n; ++j)
        cc += (colX[j] - b[j]) * (colX[j] - b[j]);
    double dp = fmax(sqrt(rr) / (1.0 + nrm2(m, a)), sqrt(cc) / (1.0 + nrm2(n, b)));
    dp = fmax(dp, sqrt(neg) / (1.0 + sqrt(xf)));
    double dc = fabs(xu) / (1.0 + sqrt(cf));

    out[0] = dphi;
    out[1] = cxh;
    out[2] = dual;
    out[3] = cx;
    out[4] = fmax(dp, dc);
    out[5] = xmin;
    out[6] = er1;
    out[7] = xu;
    out[8] = dual_g;
    out[9] = dual_p;
    if (z_out)
        memcpy(z_out, z, sizeof(double) * m);
    if (y_out)
        memcpy(y_out, y, sizeof(double) * n);
    if (er_out)
        memcpy(er_out, er, sizeof(double) * m);
    if (ec_out)
        memcpy(ec_out, ec, sizeof(double) * n);
    free(z); free(er); free(colX); free(y); free(ec); free(zc);
}

int orc_stop(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, int64_t k, double eta,
             const double *w, const double *wl, const double *gamma, const double *a, const double *b,
             const double *M, const double *S, double *out, double *xhat /* m*n or NULL */)
{
    const double sigma = (double)(k + 1) / eta;
    double *X = malloc(sizeof(double) * (size_t)m * n);
    double *logX = malloc(sizeof(double) * (size_t)m * n);
    double *psi = malloc(sizeof(double) * n);

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double la = log(a[i]), ls = log(S[i]);
        for (int64_t j = 0; j < n; ++j) {
            double x = xval(C, kind, ldc, i, j, sigma, w, wl, M[i]);
            X[i * n + j] = a[i] * (exp(x) / S[i]);
            logX[i * n + j] = la + x - ls;
        }
    }
    for (int64_t j = 0; j < n; ++j)
        psi[j] = ((wl ? w[j] + wl[j] : w[j]) - log(b[j])) / sigma;
    stop_from_plan(m, n, C, kind, ldc, X, logX, gamma, psi, a, b, out, xhat, NULL, NULL, NULL,
                   NULL);
    free(X); free(logX); free(psi);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Sinkhorn gamma-step (Algorithm 2, steps 3-4; eqs. (4)-(5) in semi-dual form):       */
/*   gamma_j += eta (log b_j - log c_j),  c_j = sum_i a_i P_ij,                         */
/* then gamma is centred.  On the potentials: w_j += log b_j - log c_j and a common     */
/* shift (which leaves P unchanged).  When some c_j is at or below the bottom of the    */
/* FP64 range (every entry of column j underflows), log c_j is taken in the log domain: */
/*   log c_j = max_i v_ij + log sum_i exp(v_ij - max_i v_ij),  v_ij = x_ij + log a_i - log S_i. */
/* ------------------------------------------------------------------------- */
static void log_colsums(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, double sigma,
                        const double *w, const double *wl, const double *a, const double *M,
                        const double *S, const double *c, double *lc)
{
    double cmin = INFINITY;
    for (int64_t j = 0; j < n; ++j)
        if (c[j] < cmin)
            cmin = c[j];
    if (!(cmin < 1e-290)) {
        for (int64_t j = 0; j < n; ++j)
            lc[j] = log(c[j]);
        return;
    }
    double *rho = malloc(sizeof(double) * m);
    for (int64_t i = 0; i < m; ++i)
        rho[i] = log(a[i]) - log(S[i]);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        double mx = -INFINITY;
        for (int64_t i = 0; i < m; ++i) {
            double v = xval(C, kind, ldc, i, j, sigma, w, wl, M[i]) + rho[i];
            if (v > mx)
                mx = v;
        }
        double sum = 0.0;
        for (int64_t i = 0; i < m; ++i)
            sum += exp((xval(C, kind, ldc, i, j, sigma, w, wl, M[i]) + rho[i]) - mx);
        lc[j] = mx + log(sum);
    }
    free(rho);
}

/* one gamma-step on the two-level potentials (w, wl) from the eval's row state (M, S) and
   column sums c at (w, wl); s is the centre's column potential (gamma = eta (w + wl - s)) */
static void sinkhorn_update(int64_t m, int64_t n, const void *C, int kind, int64_t ldc,
                            int64_t k, double eta, double q, double *w, double *wl,
                            const double *s, const double *a, const double *b, const double *M,
                            const double *S, const double *c)
{
    const double sigma = (double)(k + 1) / eta;
    double *lc = malloc(sizeof(double) * n);
    log_colsums(m, n, C, kind, ldc, sigma, w, wl, a, M, S, c, lc);
    for (int64_t j = 0; j < n; ++j)
        pot_add(&w[j], &wl[j], log(b[j]) - lc[j], q);
    /* step 4: centre gamma by a common shift of w */
    double mean = 0.0;
    for (int64_t j = 0; j < n; ++j)
        mean += eta * ((w[j] - s[j]) + wl[j]);
    mean /= (double)n;
    for (int64_t j = 0; j < n; ++j)
        pot_add(&w[j], &wl[j], -(mean / eta), q);
    free(lc);
}

/* Exported step: gamma_out = the Sinkhorn step from gamma at the centre (k, s) on the grid q,
   given the eval's row state (M, S) and column sums c at gamma. */
int orc_sinkhorn_step(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, int64_t k,
                      double eta, double q, const double *s, const double *gamma, const double *a,
                      const double *b, const double *M, const double *S, const double *c,
                      double *gamma_out)
{
    double *w = malloc(sizeof(double) * n), *wl = malloc(sizeof(double) * n);
    orc_make_w(n, s, gamma, eta, q, w, wl);
    sinkhorn_update(m, n, C, kind, ldc, k, eta, q, w, wl, s, a, b, M, S, c);
    for (int64_t j = 0; j < n; ++j)
        gamma_out[j] = eta * ((w[j] - s[j]) + wl[j]);
    free(w); free(wl);
    return ORC_OK;
}

/* Outer update (Algorithm 2, step 13 with eq. (7)): X^{k+1} = diag(a) P(gamma), i.e.
   r_i = log a_i - (M_i + log S_i) and s_j = s_j + gamma_j / eta (one double), k + 1. */
void orc_outer_update(int64_t m, int64_t n, double eta, double q, const double *a,
                      const double *M, const double *S, const double *s, const double *gamma,
                      double *r_out, double *s_out)
{
    double *w = malloc(sizeof(double) * n), *wl = malloc(sizeof(double) * n);
    orc_make_w(n, s, gamma, eta, q, w, wl);
    for (int64_t i = 0; i < m; ++i)
        r_out[i] = log(a[i]) - (M[i] + log(S[i]));
    for (int64_t j = 0; j < n; ++j)
        s_out[j] = w[j] + wl[j];
    free(w); free(wl);
}

/* ------------------------------------------------------------------------- */
/* Full IBSN (Algorithm 2) with the practical schedule of Section 5 "Setup".        */
/* ------------------------------------------------------------------------- */
typedef struct {
    double sigma_armijo, beta;        /* 1e-4, 0.8 */
    double sinkhorn_tol;              /* 1e-3 */
    int sinkhorn_maxit;               /* 10000 */
    double mu0, mu_floor;             /* 1e-4, 1e-11 */
    double gap_tol, marg_tol, kkt_tol; /* 1e-8, 1e-9, 0 (off) */
    int max_outer, max_newton, max_backtrack, cg_maxit; /* cg_maxit <= 0 -> min(n, 70) */
    double cg_forcing_max;            /* 0.1 */
    int rho_mode;                     /* 0 paper rule, 1 rho = 0 (no sparsification) */
    double cg_rtol_min;               /* 1e-6: floor of the CG relative residual */
    int stall_limit;                  /* 1 failed D_phi test after the gate ends the inner loop */
    int eot;                          /* 1: (E)IBSN of appendix C.4: centre 1 1^T, one subproblem */
    double eot_tol;                   /* (E)IBSN stops at ||g|| < eot_tol (1e-9, appendix C.4) */
    int armijo_warm;                  /* 1: each line search starts at min(1, t_prev / beta),
                                         t_prev the last accepted step; 0: at t = 1 */
} orc_options;

typedef struct {
    int64_t outer, newton, cg, sinkhorn, backtracks, stop_tests;
    double grad_norm, primal, dual, rel_gap, kkt, dphi, marg_l1;
    int status;
} orc_report;

void orc_default_options(orc_options *o)
{
    o->sigma_armijo = 1e-4;
    o->beta = 0.8;
    o->sinkhorn_tol = 1e-3;
    o->sinkhorn_maxit = 10000;
    o->mu0 = 1e-4;
    o->mu_floor = 1e-11;
    o->gap_tol = 1e-8;
    o->marg_tol = 1e-9;
    o->kkt_tol = 0.0;
    o->max_outer = 300;
    o->max_newton = 1000;
    o->max_backtrack = 60;
    o->cg_maxit = 0;
    o->cg_forcing_max = 0.1;
    o->rho_mode = 0;
    o->cg_rtol_min = 1e-6;
    o->stall_limit = 1;
    o->eot = 0;
    o->eot_tol = 1e-9;
    o->armijo_warm = 1;
}

static double nrm1(int64_t n, const double *x)
{
    double acc = 0.0;
    for (int64_t j = 0; j < n; ++j)
        acc += fabs(x[j]);
    return acc;
}

static void center(int64_t n, double *gamma)
{
    double mean = 0.0;
    for (int64_t j = 0; j < n; ++j)
        mean += gamma[j];
    mean /= (double)n;
    for (int64_t j = 0; j < n; ++j)
        gamma[j] -= mean;
}

/* gamma = eta (w + wl - s) */
static void gamma_of(int64_t n, const double *w, const double *wl, const double *s, double eta,
                     double *gamma)
{
    for (int64_t j = 0; j < n; ++j)
        gamma[j] = eta * ((w[j] - s[j]) + wl[j]);
}

/* gamma_io: in = warm start (or NULL -> 0), out = final dual.
   r_io, s_io, k_io: optional outer state (resume when *k_io > 0 and r_io, s_io given).
   plan_out: rounded plan Xhat (m*n) or NULL.  trace: optional per-outer log
   [outer][6] = {newton, cg, rel_gap, grad_norm, dphi, kkt}. */
int orc_solve(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, const double *a,
              const double *b, double eta, const orc_options *opt_in, double *gamma_io,
              double *r_io, double *s_io, int64_t *k_io, double *plan_out, orc_report *rep,
              double *trace, int64_t trace_cap)
{
    if (m < 1 || n < 1 || !(eta > 0))
        return ORC_ERR_ARG;
    orc_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        orc_default_options(&opt);
    int cg_maxit = opt.cg_maxit > 0 ? opt.cg_maxit : (int)(n < 70 ? n : 70);

    double *r = malloc(sizeof(double) * m), *s = malloc(sizeof(double) * n);
    double *gamma = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    double *wl = malloc(sizeof(double) * n);
    double *M = malloc(sizeof(double) * m), *S = malloc(sizeof(double) * m);
    double *c = malloc(sizeof(double) * n), *g = malloc(sizeof(double) * n);
    double *Mt = malloc(sizeof(double) * m), *St = malloc(sizeof(double) * m);
    double *ct = malloc(sizeof(double) * n), *gt = malloc(sizeof(double) * n);
    double *Delta = malloc(sizeof(double) * n), *rhs = malloc(sizeof(double) * n);
    double *tau = malloc(sizeof(double) * n), *d = malloc(sizeof(double) * n);
    double *lb = malloc(sizeof(double) * n);
    int64_t *row_ptr = malloc(sizeof(int64_t) * (m + 1));
    int64_t k = 0;
    if (k_io && *k_io > 0 && r_io && s_io) {
        k = *k_io;
        memcpy(r, r_io, sizeof(double) * m);
        memcpy(s, s_io, sizeof(double) * n);
    } else if (opt.eot) {
        /* (E)IBSN: X^0 = 1 1^T (appendix C.4), so the subproblem is entropic OT with cost C */
        for (int64_t i = 0; i < m; ++i)
            r[i] = 0.0;
        for (int64_t j = 0; j < n; ++j)
            s[j] = 0.0;
    } else {
        for (int64_t i = 0; i < m; ++i)
            r[i] = log(a[i]);
        for (int64_t j = 0; j < n; ++j)
            s[j] = log(b[j]);
    }
    for (int64_t j = 0; j < n; ++j) {
        gamma[j] = gamma_io ? gamma_io[j] : 0.0;
        lb[j] = log(b[j]);
    }
    if (k == 0)
        center(n, gamma); /* Lemma 4.1 needs 1^T gamma^{0,0} = 0; a resumed state already has it */

    int64_t istar = 0;
    for (int64_t i = 1; i < m; ++i)
        if (a[i] > a[istar])
            istar = i;
    const double cmax = orc_cost_max(m, n, C, kind, ldc);

    orc_report R;
    memset(&R, 0, sizeof(R));
    R.status = ORC_WARN_MAXITER;
    double stop_out[10] = {0};
    int64_t k0 = k;
    double t_prev = 1.0; /* step of the last accepted line search (armijo_warm) */
    for (; k < k0 + opt.max_outer; ++k) {
        double mu = fmax(opt.mu0 / ((double)(k + 1) * (double)(k + 1)), opt.mu_floor);
        const double q = orc_center_quantum(n, s, gamma, eta, k, cmax);
        orc_make_w(n, s, gamma, eta, q, w, wl);
        /* Algorithm 2, step 3: Sinkhorn warm-up (semi-dual form: the zeta-step is the row
           LSE of the eval pass, the gamma-step rescales the columns to b) */
        orc_eval(m, n, C, kind, ldc, k, eta, q, w, wl, NULL, NULL, a, b, M, S, c, g, NULL, NULL);
        for (int it = 0; it < opt.sinkhorn_maxit && nrm2(n, g) >= opt.sinkhorn_tol; ++it) {
            /* gamma_j += eta (log b_j - log c_j), then centred (steps 3-4) */
            sinkhorn_update(m, n, C, kind, ldc, k, eta, q, w, wl, s, a, b, M, S, c);
            orc_eval(m, n, C, kind, ldc, k, eta, q, w, wl, NULL, NULL, a, b, M, S, c, g, NULL,
                     NULL);
            ++R.sinkhorn;
        }
        /* a column whose kernel entries all lie below the FP64 range gives c_j = 0 and a
           non-finite gradient: no step can follow, report it (as the GPU solver does) */
        if (!isfinite(nrm2(n, g))) {
            R.status = ORC_ERR_NUMERIC;
            break;
        }
        int stopped = 0, stalls = 0;
        int64_t newton_k = 0, cg_k = 0;
        for (int v = 0; v < opt.max_newton; ++v) {
            double gn = nrm2(n, g);
            if (opt.eot && gn < opt.eot_tol) { /* (E)IBSN: the single subproblem is solved */
                stopped = 1;
                break;
            }
            double rho = opt.rho_mode == 1 ? 0.0 : eta * gn / ((double)m * (double)n); /* step 6 */
            int64_t nnz = orc_sparsify(m, n, C, kind, ldc, k, eta, w, wl, a, M, S, rho, istar, 0,
                                       row_ptr, NULL, NULL, NULL);
            nnz = -nnz - 1;
            int32_t *col = malloc(sizeof(int32_t) * (nnz > 0 ? nnz : 1));
            double *val = malloc(sizeof(double) * (nnz > 0 ? nnz : 1));
            orc_sparsify(m, n, C, kind, ldc, k, eta, w, wl, a, M, S, rho, istar, nnz, row_ptr,
                         col, val, d); /* step 7 */
            for (int64_t j = 0; j < n; ++j)
                rhs[j] = -g[j];
            double tol = fmax(fmin(opt.cg_forcing_max, gn), opt.cg_rtol_min) * gn;
            int it = orc_cg(m, n, row_ptr, col, val, d, a, eta, gn, rhs, tol, cg_maxit,
                            Delta); /* step 8 */
            cg_k += it;
            free(col);
            free(val);
            double gd = dot(n, g, Delta);
            double t = opt.armijo_warm ? fmin(1.0, t_prev / opt.beta) : 1.0, dL = 0.0;
            int bt = 0, accepted = 0;
            for (;;) { /* step 9: Armijo backtracking on a finite decrease */
                orc_trial(m, n, C, kind, ldc, k, eta, q, w, wl, a, b, M, Delta, t, &dL, tau, Mt,
                          St, ct, gt);
                if (isfinite(dL) && dL <= opt.sigma_armijo * t * gd) {
                    accepted = 1;
                    break;
                }
                if (bt >= opt.max_backtrack)
                    break;
                t *= opt.beta;
                ++bt;
            }
            R.backtracks += bt;
            if (!accepted) /* no acceptable step: keep the iterate and end the inner loop */
                break;
            t_prev = t;
            for (int64_t j = 0; j < n; ++j) /* step 10: w += tau, exactly */
                pot_add(&w[j], &wl[j], tau[j], q);
            memcpy(M, Mt, sizeof(double) * m);
            memcpy(S, St, sizeof(double) * m);
            memcpy(c, ct, sizeof(double) * n);
            memcpy(g, gt, sizeof(double) * n);
            ++newton_k;
            /* step 12 with the practical schedule: gradient gate, then D_phi test */
            if (!opt.eot && nrm2(n, g) < mu) {
                gamma_of(n, w, wl, s, eta, gamma);
                orc_stop(m, n, C, kind, ldc, k, eta, w, wl, gamma, a, b, M, S, stop_out, NULL);
                ++R.stop_tests;
                if (stop_out[0] <= (double)(m < n ? m : n) * mu) {
                    stopped = 1;
                    break;
                }
                if (++stalls >= opt.stall_limit)
                    break;
            }
        }
        gamma_of(n, w, wl, s, eta, gamma);
        if (!stopped || opt.eot) {
            orc_stop(m, n, C, kind, ldc, k, eta, w, wl, gamma, a, b, M, S, stop_out, NULL);
            ++R.stop_tests;
        }
        R.newton += newton_k;
        R.cg += cg_k;
        double primal = stop_out[1], dual = stop_out[2];
        double relgap = (primal - dual) / fabs(primal);
        double marg = nrm1(n, g);
        if (trace && (k - k0) < trace_cap) {
            double *tr = trace + (k - k0) * 6;
            tr[0] = (double)newton_k;
            tr[1] = (double)cg_k;
            tr[2] = relgap;
            tr[3] = nrm2(n, g);
            tr[4] = stop_out[0];
            tr[5] = stop_out[4];
        }
        R.primal = primal;
        R.dual = dual;
        R.rel_gap = relgap;
        R.kkt = stop_out[4];
        R.dphi = stop_out[0];
        R.grad_norm = nrm2(n, g);
        R.marg_l1 = marg;
        int done = (relgap <= opt.gap_tol && (opt.marg_tol <= 0 || marg <= opt.marg_tol)) ||
                   (opt.kkt_tol > 0 && stop_out[4] <= opt.kkt_tol);
        if (opt.eot) {
            /* (E)IBSN: one subproblem, no outer update; done when its gradient is small */
            if (plan_out)
                orc_stop(m, n, C, kind, ldc, k, eta, w, wl, gamma, a, b, M, S, stop_out, plan_out);
            R.status = R.grad_norm < opt.eot_tol ? ORC_OK : ORC_WARN_MAXITER;
            ++k; /* one subproblem solved; the centre (r, s) = (0, 0) is left as it was */
            break;
        }
        if (plan_out && (done || k + 1 == k0 + opt.max_outer))
            orc_stop(m, n, C, kind, ldc, k, eta, w, wl, gamma, a, b, M, S, stop_out, plan_out);
        /* Algorithm 2, step 13: X^{k+1} = X^{k,v+1}: r = log a - lse, s = w, k = k+1;
           gamma^{k+1,0} = gamma^{k,v+1} */
        for (int64_t i = 0; i < m; ++i)
            r[i] = log(a[i]) - (M[i] + log(S[i]));
        /* s = w rounded to one double: a column rescaling of X^{k+1} by 1 + O(2^-53), which
           the next subproblem's dual absorbs (its optimal plan is unchanged) */
        for (int64_t j = 0; j < n; ++j)
            s[j] = w[j] + wl[j];
        if (done) {
            R.status = ORC_OK;
            ++k;
            break;
        }
    }
    R.outer = k - k0;
    if (gamma_io)
        memcpy(gamma_io, gamma, sizeof(double) * n);
    if (r_io)
        memcpy(r_io, r, sizeof(double) * m);
    if (s_io)
        memcpy(s_io, s, sizeof(double) * n);
    if (k_io)
        *k_io = k;
    if (rep)
        *rep = R;
    free(r); free(s); free(gamma); free(w); free(wl); free(M); free(S); free(c); free(g); free(Mt);
    free(St); free(ct); free(gt); free(Delta); free(rhs); free(tau); free(d); free(lb);
    free(row_ptr);
    return R.status;
}

/* ========================================================================= */
/* Plain reference passes.  The same quantities as orc_eval, orc_sparsify and      */
/* orc_stop, taken straight from their definitions with no potential grid:          */
/*   w_j = s_j + gamma_j/eta,  theta_ij = fma(-sigma, C_ij, w_j),  sigma = (k+1)/eta  */
/* (eq. (7) with the implicit centre log X^k_ij = r_i + s_j - k C_ij/eta: the row     */
/* term r_i cancels in P), M_i = max_j theta_ij, S_i = sum_j exp(theta_ij - M_i),     */
/* lse_i = M_i + log S_i (eq. (5) up to the row constant), and                        */
/*   P_ij = exp(theta_ij - lse_i), evaluated as exp(theta_ij - M_i) / S_i,            */
/* which is the same number in exact arithmetic and does not round lse_i at the       */
/* scale of sigma.  These functions are the definition the HIP passes are held to;   */
/* the grid functions above are the solver's own scheme and are held to these too.   */
/* ========================================================================= */

/* theta of row i at the plain potentials w; returns M_i and S_i */
static void plain_row(const void *C, int kind, int64_t ldc, int64_t i, int64_t n, double sigma,
                      const double *w, double *theta, double *Mi, double *Si)
{
    double mx = -INFINITY;
    for (int64_t j = 0; j < n; ++j) {
        theta[j] = fma(-sigma, cost_at(C, kind, ldc, i, j), w[j]);
        if (theta[j] > mx)
            mx = theta[j];
    }
    double sum = 0.0;
    for (int64_t j = 0; j < n; ++j)
        sum += exp(theta[j] - mx);
    *Mi = mx;
    *Si = sum;
}

static void plain_w(int64_t n, const double *s, const double *gamma, double eta, double *w)
{
    for (int64_t j = 0; j < n; ++j)
        w[j] = s[j] + gamma[j] / eta;
}

/* Eval (eqs. (5)-(8)): lse (m), c = P^T a, g = c - b (n), L (eq. (6)), plan = diag(a) P.
   r may be NULL (then L is not formed); lse and plan may be NULL. */
int orc_plain_eval(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, int64_t k,
                   double eta, const double *r, const double *s, const double *gamma,
                   const double *a, const double *b, double *lse, double *c, double *g, double *L,
                   double *plan)
{
    if (m < 1 || n < 1 || !(eta > 0))
        return ORC_ERR_ARG;
    const double sigma = (double)(k + 1) / eta;
    double *w = malloc(sizeof(double) * n);
    double *Mv = malloc(sizeof(double) * m), *Sv = malloc(sizeof(double) * m);
    plain_w(n, s, gamma, eta, w);
    double *part = calloc((size_t)ORC_NCHUNK * n, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int qq = 0; qq < ORC_NCHUNK; ++qq) {
        int64_t i0 = m * qq / ORC_NCHUNK, i1 = m * (qq + 1) / ORC_NCHUNK;
        double *pc = part + (size_t)qq * n;
        double *theta = malloc(sizeof(double) * n);
        for (int64_t i = i0; i < i1; ++i) {
            plain_row(C, kind, ldc, i, n, sigma, w, theta, &Mv[i], &Sv[i]);
            for (int64_t j = 0; j < n; ++j) {
                double p = exp(theta[j] - Mv[i]) / Sv[i];
                pc[j] += a[i] * p;
                if (plan)
                    plan[i * n + j] = a[i] * p;
            }
        }
        free(theta);
    }
    for (int64_t j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int qq = 0; qq < ORC_NCHUNK; ++qq)
            acc += part[(size_t)qq * n + j];
        c[j] = acc;
        g[j] = acc - b[j];
    }
    free(part);
    if (lse)
        for (int64_t i = 0; i < m; ++i)
            lse[i] = Mv[i] + log(Sv[i]);
    if (L && r) {
        double t = 0.0;
        for (int64_t i = 0; i < m; ++i)
            t += a[i] * (r[i] + (Mv[i] + log(Sv[i])));
        *L = -dot(n, b, gamma) + eta * t;
    }
    free(w); free(Mv); free(Sv);
    return ORC_OK;
}

/* Algorithm 1 on the plain P at (k, s, gamma): rows i != istar keep P_ij >= rho and are
   divided by their kept sum; row istar is kept whole.  CSR in row order, columns
   ascending, d = P_rho^T a.  Returns nnz, or -(needed nnz) - 1 when cap is too small
   (then only row_ptr is written). */
int64_t orc_plain_sparsify(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, int64_t k,
                           double eta, const double *s, const double *gamma, const double *a,
                           double rho, int64_t istar, int64_t cap, int64_t *row_ptr, int32_t *col,
                           double *val, double *d)
{
    const double sigma = (double)(k + 1) / eta;
    double *w = malloc(sizeof(double) * n);
    plain_w(n, s, gamma, eta, w);
    double *P = malloc(sizeof(double) * (size_t)m * n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double Mi, Si;
        double *theta = P + (size_t)i * n;
        plain_row(C, kind, ldc, i, n, sigma, w, theta, &Mi, &Si);
        for (int64_t j = 0; j < n; ++j)
            theta[j] = exp(theta[j] - Mi) / Si;
    }
    row_ptr[0] = 0;
    for (int64_t i = 0; i < m; ++i) {
        int64_t cnt = 0;
        for (int64_t j = 0; j < n; ++j)
            if (i == istar || P[(size_t)i * n + j] >= rho)
                ++cnt;
        row_ptr[i + 1] = row_ptr[i] + cnt;
    }
    int64_t nnz = row_ptr[m];
    if (nnz > cap) {
        free(w); free(P);
        return -nnz - 1;
    }
    for (int64_t i = 0; i < m; ++i) {
        int64_t o = row_ptr[i];
        double kappa = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double p = P[(size_t)i * n + j];
            if (i == istar || p >= rho) {
                col[o] = (int32_t)j;
                val[o] = p;
                kappa += p;
                ++o;
            }
        }
        if (i != istar && kappa > 0.0)
            for (int64_t e = row_ptr[i]; e < o; ++e)
                val[e] = val[e] / kappa;
    }
    for (int64_t j = 0; j < n; ++j)
        d[j] = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            d[col[e]] += a[i] * val[e];
    free(w); free(P);
    return nnz;
}

/* Algorithm 3, D_phi(Xhat, X) (eq. (3), log domain) and the certificate of orc_stop for the
   plain plan X = diag(a) P at (k, s, gamma); log X_ij = log a_i + (theta_ij - M_i) - log S_i;
   psi_j = (w_j - log b_j)/sigma with the plain w.  Optional outputs: xhat (m*n), z, e_r (m),
   y, e_c (n) of Algorithm 3. */
int orc_plain_stop(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, int64_t k,
                   double eta, const double *s, const double *gamma, const double *a,
                   const double *b, double *out, double *xhat, double *z, double *y, double *er,
                   double *ec)
{
    const double sigma = (double)(k + 1) / eta;
    double *w = malloc(sizeof(double) * n), *psi = malloc(sizeof(double) * n);
    double *X = malloc(sizeof(double) * (size_t)m * n);
    double *logX = malloc(sizeof(double) * (size_t)m * n);
    plain_w(n, s, gamma, eta, w);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double Mi, Si;
        double *theta = X + (size_t)i * n;
        plain_row(C, kind, ldc, i, n, sigma, w, theta, &Mi, &Si);
        const double la = log(a[i]), ls = log(Si);
        for (int64_t j = 0; j < n; ++j) {
            const double x = theta[j] - Mi;
            logX[(size_t)i * n + j] = la + x - ls;
            theta[j] = a[i] * (exp(x) / Si);
        }
    }
    for (int64_t j = 0; j < n; ++j)
        psi[j] = (w[j] - log(b[j])) / sigma;
    stop_from_plan(m, n, C, kind, ldc, X, logX, gamma, psi, a, b, out, xhat, z, y, er, ec);
    free(w); free(psi); free(X); free(logX);
    return ORC_OK;
}
