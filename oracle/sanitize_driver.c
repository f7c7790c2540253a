/* sanitize_driver.c -- runs the oracle's solver and plain passes on small problems, built
 * with AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py
 * (test infrastructure only).  Every solver phase (Sinkhorn warm-up, eval, sparsify, CG,
 * Armijo trials, the stop test with Algorithm 3, the outer update) runs on each case;
 * a sanitizer report or a failed status exits non-zero. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    double sigma_armijo, beta, sinkhorn_tol;
    int sinkhorn_maxit;
    double mu0, mu_floor, gap_tol, marg_tol, kkt_tol;
    int max_outer, max_newton, max_backtrack, cg_maxit;
    double cg_forcing_max;
    int rho_mode;
    double cg_rtol_min;
    int stall_limit, eot;
    double eot_tol;
    int armijo_warm;
} orc_options;
typedef struct {
    int64_t outer, newton, cg, sinkhorn, backtracks, stop_tests;
    double grad_norm, primal, dual, rel_gap, kkt, dphi, marg_l1;
    int status;
} orc_report;

void orc_default_options(orc_options *o);
int orc_solve(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, const double *a,
              const double *b, double eta, const orc_options *opt, double *gamma_io,
              double *r_io, double *s_io, int64_t *k_io, double *plan_out, orc_report *rep,
              double *trace, int64_t trace_cap);
int orc_plain_eval(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, int64_t k,
                   double eta, const double *r, const double *s, const double *gamma,
                   const double *a, const double *b, double *lse, double *c, double *g, double *L,
                   double *plan);
int orc_plain_stop(int64_t m, int64_t n, const void *C, int kind, int64_t ldc, int64_t k,
                   double eta, const double *s, const double *gamma, const double *a,
                   const double *b, double *out, double *xhat, double *z, double *y, double *er,
                   double *ec);

static uint64_t st = 88172645463325252ull;
static double urand(void)   /* xorshift64, uniform in (0, 1) */
{
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return ((double)(st >> 11) + 0.5) / 9007199254740992.0;
}

static int run(int64_t m, int64_t n, double eta, int rho_mode, int eot, int f32)
{
    double *C = malloc(sizeof(double) * m * n), *a = malloc(sizeof(double) * m);
    float *Cf = malloc(sizeof(float) * m * n);
    double *b = malloc(sizeof(double) * n), *gamma = calloc(n, sizeof(double));
    double *plan = malloc(sizeof(double) * m * n), *trace = malloc(sizeof(double) * 6 * 64);
    double sa = 0.0, sb = 0.0, cmax = 0.0;
    for (int64_t i = 0; i < m * n; ++i) {
        C[i] = urand();
        cmax = C[i] > cmax ? C[i] : cmax;
    }
    for (int64_t i = 0; i < m * n; ++i) {
        C[i] /= cmax;
        Cf[i] = (float)C[i];
    }
    for (int64_t i = 0; i < m; ++i)
        sa += (a[i] = 0.5 + urand());
    for (int64_t j = 0; j < n; ++j)
        sb += (b[j] = 0.5 + urand());
    for (int64_t i = 0; i < m; ++i)
        a[i] /= sa;
    for (int64_t j = 0; j < n; ++j)
        b[j] /= sb;
    orc_options o;
    orc_default_options(&o);
    o.max_outer = 40;
    o.rho_mode = rho_mode;
    o.eot = eot;
    orc_report rep;
    const int rc = orc_solve(m, n, f32 ? (const void *)Cf : (const void *)C, f32, n, a, b, eta,
                             &o, gamma, NULL, NULL, NULL, plan, &rep, trace, 64);
    int bad = rc < 0 || !(rep.primal == rep.primal);
    /* plain passes at the final dual (k = 0 centre r = log a, s = log b) */
    double *r = malloc(sizeof(double) * m), *s = malloc(sizeof(double) * n);
    double *lse = malloc(sizeof(double) * m), *c = malloc(sizeof(double) * n);
    double *g = malloc(sizeof(double) * n), L = 0.0, out[16];
    double *z = malloc(sizeof(double) * m), *y = malloc(sizeof(double) * n);
    double *er = malloc(sizeof(double) * m), *ec = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < m; ++i)
        r[i] = log(a[i]);
    for (int64_t j = 0; j < n; ++j)
        s[j] = log(b[j]);
    bad |= orc_plain_eval(m, n, C, 0, n, 0, eta, r, s, gamma, a, b, lse, c, g, &L, plan) < 0;
    bad |= orc_plain_stop(m, n, C, 0, n, 0, eta, s, gamma, a, b, out, plan, z, y, er, ec) < 0;
    printf("m %lld n %lld eta %g rho_mode %d eot %d f32 %d: rc %d outer %lld newton %lld "
           "gap %.3g\n", (long long)m, (long long)n, eta, rho_mode, eot, f32, rc,
           (long long)rep.outer, (long long)rep.newton, rep.rel_gap);
    free(C); free(Cf); free(a); free(b); free(gamma); free(plan); free(trace);
    free(r); free(s); free(lse); free(c); free(g); free(z); free(y); free(er); free(ec);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= run(13, 11, 0.1, 0, 0, 0);
    bad |= run(7, 19, 0.02, 0, 0, 0);
    bad |= run(16, 16, 0.05, 1, 0, 0);
    bad |= run(9, 12, 0.05, 0, 1, 0);
    bad |= run(12, 10, 0.1, 0, 0, 1);
    bad |= run(1, 5, 0.1, 0, 0, 0);
    bad |= run(5, 1, 0.1, 0, 0, 0);
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
