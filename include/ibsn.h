/*
 * ibsn.h -- C ABI of libibsn.so, the MI355X (gfx950) hot path of the Inexact
 * Bregman Sparse Newton (IBSN) method for exact optimal transport.
 *
 * The problem (eq. (1)) is   min <C,X>  s.t.  X 1 = a,  X^T 1 = b,  X >= 0,
 * with C >= 0 (m x n), a > 0 (m), b > 0 (n), 1^T a = 1^T b = 1.  IBSN solves it by
 * the Bregman proximal point iteration of eq. (3) and Algorithm 2; each proximal
 * subproblem is solved in its semi-dual form (eq. (6)) by a Sinkhorn warm-up and a
 * sparsified (Algorithm 1), gradient-shifted Newton-CG method with Armijo steps.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array pointers are DEVICE pointers (HIP, the context's device) unless the
 *    argument is marked "host".  All floating point arrays are IEEE FP64, C order.
 *  - The caller owns every array it passes (inputs and outputs); the library never
 *    frees them.  The library owns its context workspace and ibsn_csr handles.
 *  - Calls are enqueued on the context's stream and are asynchronous, except that a
 *    call returning a host value (marked "host out") synchronises that stream.
 *  - One context per host thread; a context may be used from one thread at a time.
 *  - Return value: IBSN_OK (0), a positive warning (results valid), or a negative
 *    error (nothing is written past the point of the error; ibsn_last_error() holds
 *    a message).
 *
 * Prox centre (row a1 of the path)
 * --------------------------------
 * X^0 = a b^T and X^{k+1} = diag(a) P^k(gamma) (eq. (7)) give, for every k,
 *     log X^k_ij = r_i + s_j - k C_ij / eta,
 * so the centre is held implicitly as (k, r, s): r = log a, s = log b at k = 0 and
 * r <- log a - lse, s <- s + gamma/eta, k <- k+1 at an outer update.  The plan of the
 * subproblem at gamma is the row softmax of theta_ij = w_j - sigma C_ij with
 * sigma = (k+1)/eta and w_j = s_j + gamma_j/eta (on the grid of ibsn_center).
 *
 * Row state
 * ---------
 * A pair of m-vectors (M, S) represents P_ij = exp(x_ij) / S_i with
 * x_ij = fma(-sigma, C_ij, w_j - M_i) = theta_ij - M_i, the plan of eq. (7) with a
 * per-row shift M_i on the grid.  ibsn_subproblem_eval() sets M_i to the grid-rounded
 * max_j theta_ij and S_i = sum_j exp(x_ij); ibsn_trial() returns the state of the trial
 * point.  lse_i = M_i + log S_i is the row log-sum-exp of eq. (5).
 */
#ifndef IBSN_H
#define IBSN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    IBSN_OK = 0,
    IBSN_WARN_MAXITER = 1,        /* ibsn_solve: max_outer reached before the stop rule */
    IBSN_ERR_INVALID_ARG = -1,    /* a size, pointer or value violates the stated contract */
    IBSN_ERR_HIP = -2,            /* a HIP runtime call failed                            */
    IBSN_ERR_OOM = -3,            /* workspace allocation failed                          */
    IBSN_ERR_NUMERIC = -4,        /* NaN or Inf met where a finite value is required       */
    IBSN_ERR_UNSUPPORTED = -5     /* shape outside the compiled kernel range               */
};

/* Widest row a dense kernel holds whole: a workgroup keeps one row of C in registers and
   an n-vector of potentials in LDS (FP64 cost and points: 10240 columns; FP32 cost: 20000).
   Wider rows are split into column blocks (ibsn_set_row_split). */
#define IBSN_MAX_N_F64 10240
#define IBSN_MAX_N_F32 20000

typedef struct ibsn_ctx ibsn_ctx;
typedef struct ibsn_csr ibsn_csr;

/* Create a context on HIP device `device` using stream `hip_stream` (a hipStream_t;
   NULL = the null stream).  Workspace is allocated lazily and grown on demand. */
int ibsn_create(ibsn_ctx **out, int device, void *hip_stream);
void ibsn_destroy(ibsn_ctx *ctx);
/* Host string describing the last error on ctx; valid until the next call on ctx. */
const char *ibsn_last_error(const ibsn_ctx *ctx);
/* Number of compute units of the context's device (host value). */
int ibsn_num_cus(const ibsn_ctx *ctx);
/* How the context runs CG (Algorithm 2, step 8; ibsn_cg and the Newton steps of the
   solvers).  IBSN_CG_PERSISTENT: every iteration inside one cooperative launch of `blocks`
   resident workgroups (0: chosen from the problem size) with two grid-wide barriers per
   iteration; IBSN_CG_LAUNCHES: three kernel launches per iteration, the host following the
   residual in chunks; IBSN_CG_SINGLE: every iteration inside one workgroup of 1024 threads
   with p and a.(P_rho p) in LDS (needs n <= 10240 and (m + n) doubles of LDS, else
   IBSN_ERR_UNSUPPORTED from the CG calls); IBSN_CG_PIPE: one cooperative launch with one
   grid-wide barrier per iteration, on M = P'^T diag(a) P' (the factor without its dense
   row, formed once per CG solve; the dense row stays a rank-one term) and the pipelined CG
   recurrences (Ghysels and Vanroose 2014); IBSN_CG_AUTO (the default): one workgroup for a
   factor of at most 3 max(m, n) stored entries with m, n <= 4096, else, with cooperative
   launches, the one-barrier form when M has at most 4 times the factor's entries plus n
   and the persistent form otherwise, else launches.  The forms run the same recurrences;
   p.(H_rho + shift I)p is taken as the quadratic form (sum d p^2 - sum a (P_rho p)^2)/eta +
   shift sum p^2 in the persistent and one-workgroup forms and as the dot product of p with
   the computed product in the other, so iterates agree to rounding.  ibsn_solve_batch with
   more than one context makes no cooperative launches (a cooperative grid assumes the
   device to itself): CG runs in one workgroup where AUTO or SINGLE takes it, else as
   launches.  IBSN_ERR_INVALID_ARG for an unknown mode or blocks outside 0..1024,
   IBSN_ERR_UNSUPPORTED for IBSN_CG_PERSISTENT or IBSN_CG_PIPE without cooperative launches; a grid larger
   than the device can hold resident makes the CG calls fail with IBSN_ERR_HIP. */
enum { IBSN_CG_AUTO = 0, IBSN_CG_LAUNCHES = 1, IBSN_CG_PERSISTENT = 2, IBSN_CG_SINGLE = 3,
       IBSN_CG_PIPE = 4 };
int ibsn_set_cg_kernel(ibsn_ctx *ctx, int mode, int blocks);
/* Rows wider than a tile (the dense passes of eq. (6)-(8), Algorithm 1 and Algorithm 3).
   cols = 0 (the default): rows of more than IBSN_MAX_N_F64 columns (FP64 cost, points) or
   IBSN_MAX_N_F32 (FP32 cost) are split into equal column blocks of at most 10240 (FP64,
   points) or 12288 (FP32) columns; cols > 0: rows of more than cols columns are split into
   blocks of at most cols columns (a multiple of 64 in [256, IBSN_MAX_N_F64]).  Each pass then
   runs its kernel per block and joins the blocks per row: the row maximum and sum of the
   eval and trial passes combine across blocks, and their column sums take a second launch
   per block (the cost is read twice); sparsify joins the blocks' kept entries per row and
   forms d from the transpose; the stop test joins its per-row sums and minima.  Results
   equal the whole-row passes to rounding.  ibsn_autotune refuses split problems.
   IBSN_ERR_INVALID_ARG for another cols. */
int ibsn_set_row_split(ibsn_ctx *ctx, int64_t cols);
/* The transpose of the sparsified factor (Algorithm 1's P_rho, read by the column products
   of Algorithm 2, step 8) is written by one of two fills with the same result, bit for bit:
   IBSN_CSC_ENTRY scatters entry by entry; IBSN_CSC_BLOCK stages blocks of 32 rows by column
   tiles in LDS and writes each column's entries of the block as one contiguous run.
   IBSN_CSC_AUTO (the default) takes the block fill once the factor stores at least m n / 32
   entries, decided on the device from the entry count.  IBSN_ERR_INVALID_ARG for another
   mode. */
enum { IBSN_CSC_AUTO = 0, IBSN_CSC_ENTRY = 1, IBSN_CSC_BLOCK = 2 };
int ibsn_set_csc_fill(ibsn_ctx *ctx, int mode);

typedef enum { IBSN_COST_F64 = 0, IBSN_COST_F32 = 1, IBSN_COST_POINTS = 2 } ibsn_cost_kind;

/* Arithmetic of the m x n passes.  IBSN_PREC_F64: everything in FP64.
   IBSN_PREC_MIXED (the precision form; the paper fixes no precision): the eval, trial and
   sparsify passes take exp(theta_ij - M_i) in FP32 (argument formed in FP64, relative
   error of each exponential about 2^-22) and the sparsified factor stores FP32 values,
   which the HVP widens to FP64; shifts, row sums, column sums, CG dot products and norms,
   the stop test with its rounding and certificate, and the objective stay FP64.  Results
   of the pass-level calls then carry relative errors of a few 1e-7 (S, c, g, plan, the
   factor's values).  An Armijo trial whose largest potential step t Delta_j / eta exceeds
   80 runs in FP64 (its unshifted factors q e^tau could exceed the FP32 range).
   ibsn_solve switches back to FP64 passes near convergence (see
   ibsn_options.mixed_switch), so its final iterate is held to FP64 accuracy. */
typedef enum { IBSN_PREC_F64 = 0, IBSN_PREC_MIXED = 1 } ibsn_precision;

/* OT problem, eq. (1).  C is row-major with leading dimension ldc >= n (elements);
   an FP32 cost is widened exactly to FP64 before use.  No rescaling of C is done:
   normalising max C to 1 (Section 5, "Setup") is the caller's job.
   Contract (checked by ibsn_solve, assumed by the pass-level calls):
   m >= 1, n >= 1, eta > 0 finite, a > 0, b > 0, |sum a - 1|, |sum b - 1| <= 1e-12*max(m,n). */
typedef struct {
    int64_t m, n;
    int32_t cost_kind;        /* ibsn_cost_kind */
    int32_t precision;        /* ibsn_precision (0 = FP64) */
    const void *C;
    int64_t ldc;
    const double *a, *b;      /* device, m and n */
    double eta;
    /* IBSN_COST_POINTS: the cost is not stored but formed from points in every pass:
       C points to x (m x dim, row-major FP64), ldc = dim (2 or 3), y (n x dim) and
       C_ij = cost_scale * ((x_i1 - y_j1)^2 + (x_i2 - y_j2)^2 [+ (x_i3 - y_j3)^2]), each
       square and sum rounded separately, in that order (no fused multiply-add), so that a
       caller can form the same matrix exactly.  Unused for the stored cost kinds. */
    const double *y;
    double cost_scale;
} ibsn_problem;

/* Tiles of the dense passes: the light tile (eval, stop test: nt threads, q vector slots
   per thread, the first qf of them inside the row), the heavy tile (trial, sparsify) and
   the grid shared by all passes. */
typedef struct {
    int32_t nt, q, qf, nt_h, q_h, qf_h, grid, reserved;
    double light_ms, heavy_ms;                 /* chosen tiles: eval + stop, trial + sparsify */
    double default_light_ms, default_heavy_ms; /* the built-in table's tiles, same timings */
} ibsn_tile;
/* Autotuner of the dense-pass tiles (NEXT-3).  Times every compiled tile that can hold a
   row of prob's n entries, on prob itself (the first subproblem's state at gamma = 0):
   light tiles on one eval and one stop test, heavy tiles on one trial pass and one
   sparsify pass, each the mean of three calls after one untimed, for grids of 1, 2 and 4
   workgroups per compute unit.  Records the fastest combination for problems of the same
   shape (m, n, cost kind, precision) on this context: later calls on the context with such
   a problem (ibsn_solve, the pass entry points) use it; results then differ from the
   default tiles' only by the order of summation.  out (host, optional): the choice and the
   timings.  prob = NULL clears the context's records.  Synchronises; allocates the
   solver's workspace for prob. */
int ibsn_autotune(ibsn_ctx *ctx, const ibsn_problem *prob, ibsn_tile *out);

/* Implicit prox centre X^k (see above): device r (m), s (n), and the grid spacing
   `quantum` (a power of two, at least DBL_MIN) of the potentials.  Every pass forms
   w_j = s_j + gamma_j/eta as two parts, wh_j = grid(s_j + gamma_j/eta) with
   grid(v) = quantum * rint(v / quantum) and the remainder wl_j (exact up to the rounding
   of gamma_j/eta), keeps the row shifts M_i on the same grid, and evaluates
   x_ij = fma(-sigma, C_ij, wh_j - M_i) + wl_j: the difference wh_j - M_i is exact, so
   x_ij = theta_ij - M_i carries two roundings at its own scale however large sigma
   grows.  (FP32 costs with n > 12288 keep the potentials on the grid: wl_j = 0, w_j =
   grid(s_j + gamma_j/eta).)  ibsn_center_quantum() returns the spacing the solver uses:
   2^(e-50) for 2^(e-1) <= max_j |s_j + gamma_j/eta| + sigma max|C| < 2^e. */
typedef struct {
    int64_t k;
    const double *r, *s;
    double quantum;
} ibsn_center;

/* Initial prox centre X^0 = a b^T (Algorithm 2 input): r = log a (m), s = log b (n),
   device outputs the caller owns; k = 0.  Asynchronous on the context's stream. */
int ibsn_center_init(ibsn_ctx *ctx, const ibsn_problem *prob, double *r, double *s);

/* Host out: the grid spacing for (prob, ctr.k, ctr.s, gamma) (see ibsn_center).
   Reads C once (max |C|).  Synchronises. */
int ibsn_center_quantum(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
                        const double *gamma, double *quantum_host);

/* Subproblem evaluation (eq. (5)-(8)): the row LSE pass over the m x n kernel.
   In: gamma (n).  Out: M, S (m) row state; lse (m, optional) = M + log S;
   colmarg (n) = P^T a; grad (n) = P^T a - b (the paper's sign; the marginal
   residual X^T 1 - b of the plan X = diag(a) P); obj_host (host out, optional)
   = L^k(gamma) of eq. (6); plan (m x n row-major, optional) = diag(a) P.
   Optional outputs may be NULL.  obj_host != NULL synchronises the stream. */
int ibsn_subproblem_eval(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
                         const double *gamma, double *M, double *S, double *lse,
                         double *colmarg, double *grad, double *obj_host, double *plan);

/* Armijo trial (Algorithm 2, step 9) from the row state (M) of gamma.  The step is
   tau_j = t Delta_j / eta (on the potential grid, grid(t Delta_j / eta), where the
   potentials are kept on it), trial point w + tau.
   Host out dL = L^k(trial) - L^k(gamma), evaluated in difference form
   (-eta b^T tau + eta sum_i a_i log(sum_j q_ij e^{tau_j} / sum_j q_ij), q = exp(x)) so
   that it keeps its relative precision for tiny steps.  Device out: M_new, S_new (m)
   row state of the trial point, colmarg_new, grad_new (n).  Synchronises. */
int ibsn_trial(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
               const double *gamma, const double *M, const double *Delta, double t,
               double *dL_host, double *M_new, double *S_new, double *colmarg_new,
               double *grad_new);

/* Sinkhorn gamma-step of the warm-up (Algorithm 2, steps 3-4), from the eval's row state
   (M, S) and column sums colmarg = P^T a at gamma: gamma_out = gamma + eta (log b - log c),
   then centred (sum_j gamma_out_j = 0; P is unchanged by the shift).  log c_j is formed in
   the log domain, by a column log-sum-exp pass over C, when some c_j < 1e-290, so that a
   column whose kernel entries all underflow still moves.  gamma_out (n) may alias gamma.
   Synchronises (one scalar read). */
int ibsn_sinkhorn_step(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
                       const double *gamma, const double *M, const double *S,
                       const double *colmarg, double *gamma_out);

/* Outer update (Algorithm 2, step 13 with eq. (7)): the next centre X^{k+1} = diag(a) P at
   gamma, from the row state (M, S) at gamma: r_out = log a - (M + log S) (m) and
   s_out = s + gamma/eta (n, the two-level potential rounded to one double: a column
   rescaling of X^{k+1} by 1 + O(2^-53), absorbed by the next subproblem's dual).  The
   caller advances k.  r_out and s_out may alias ctr->r and ctr->s. */
int ibsn_outer_update(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
                      const double *gamma, const double *M, const double *S, double *r_out,
                      double *s_out);

/* Hessian sparsification, Algorithm 1, from the row state (M, S) at gamma:
   P_ij = exp(x_ij)/S_i; rows i != istar keep P_ij >= rho (inclusive) divided
   by their kept sum; row istar is kept whole.  istar < 0 selects argmax a (lowest
   index on ties).  *out receives a library-owned handle (free with ibsn_csr_free);
   it also holds d = P_rho^T a and the transpose used by ibsn_hvp.  A row whose
   entries all fall below rho is left empty.  ibsn_destroy releases the device memory of
   the handles of its context that are still open; such a handle is then valid only for
   ibsn_csr_free (which frees what remains), and the calls that take it with a context
   return IBSN_ERR_INVALID_ARG for it, as for a handle of another context.
   IBSN_PREC_MIXED: the values are stored as FP32 (P~) and d = P~^T (a o P~ 1), so that
   H_rho 1 = 0 and H_rho is positive semidefinite for the stored factor (Theorem 3.2);
   P~ 1 = 1 up to FP32 rounding of the values.  Needs 24*m*n bytes of workspace. */
int ibsn_sparsify(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
                  const double *gamma, const double *M, const double *S, double rho,
                  int64_t istar, ibsn_csr **out);

/* Host out: nnz and istar of a sparsified factor (synchronises). */
int ibsn_csr_info(ibsn_ctx *ctx, const ibsn_csr *csr, int64_t *nnz, int64_t *istar);

/* Copy the factor out as standard CSR in row order, columns ascending:
   row_ptr (m+1, int64), col (nnz, int32), val (nnz), d (n) -- device buffers the
   caller sized from ibsn_csr_info. */
int ibsn_csr_export(ibsn_ctx *ctx, const ibsn_csr *csr, int64_t *row_ptr, int32_t *col,
                    double *val, double *d);
void ibsn_csr_free(ibsn_csr *csr);

/* Sparse Hessian-vector product (Algorithm 1, step 4 and Algorithm 2, step 8):
   y = (diag(P_rho^T a) v - P_rho^T diag(a) P_rho v)/eta + shift*v, for v, y in R^n.
   H_rho is never formed.  a must be the problem's a (m). */
int ibsn_hvp(ibsn_ctx *ctx, const ibsn_csr *csr, const double *a, double eta, double shift,
             const double *v, double *y);

/* ibsn_hvp for callers that cannot allocate device memory (code under HIP graph capture,
   tight serving loops, harnesses that forbid allocation): the same product and kernels,
   but no allocation of any kind.  The intermediate u = a o (P_rho v) (m doubles) and the
   dense row's partial sums go to one fixed device array of the library, about 8 MiB per
   device, located by ibsn_create and held until the process ends.  Requires m <=
   IBSN_NOALLOC_MAX_M (else IBSN_ERR_INVALID_ARG, nothing launched).  Every call on one
   device uses that device's array: calls that overlap on one device (other streams, other
   threads, other contexts) race and must be serialised by the caller.  The array needs no
   clearing: each call writes every entry it reads before reading it. */
#define IBSN_NOALLOC_MAX_M 1048576
int ibsn_hvp_noalloc(ibsn_ctx *ctx, const ibsn_csr *csr, const double *a, double eta,
                     double shift, const double *v, double *y);

/* Conjugate gradients (Algorithm 2, step 8) for (H_rho + shift I) x = rhs from x = 0,
   stopping at ||r||_2 <= tol or after maxit iterations.  Host out: iterations. */
int ibsn_cg(ibsn_ctx *ctx, const ibsn_csr *csr, const double *a, double eta, double shift,
            const double *rhs, double tol, int maxit, double *x, int *iters_host);

/* Inexact stop test and certificate for the plan X = diag(a) P of the row state (M, S):
   Algorithm 3 rounding, D_phi(Xhat, X) (eq. (3)), <C,Xhat>, and the dual lower bound
   max over v in {gamma, psi} of a^T zeta^c(v) + b^T v with zeta^c_i = min_j (C_ij - v_j)
   (the c-transform of appendix C.1) and psi_j = (w_j - log b_j)/sigma.
   Host out (10 values): [0] D_phi, [1] <C,Xhat>, [2] best dual bound, [3] <C,X>,
   [4] Delta_kkt (appendix C.1, for (X, gamma, zeta^c(gamma))), [5] min Xhat,
   [6] ||e_r||_1, [7] <X, U(gamma, zeta^c)>, [8] bound from gamma, [9] bound from psi.
   xhat (m x n, optional) receives the rounded plan.  Synchronises. */
int ibsn_stop(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_center *ctr,
              const double *gamma, const double *M, const double *S, double *out_host,
              double *xhat);

/* Kernel timing with HIP events recorded on the context's stream around the main
   kernel of each phase.  ibsn_kernel_timing(ctx, 1) enables it and clears the totals;
   0 disables it.  ibsn_kernel_times_get() (host out, synchronises) returns, per phase,
   the summed kernel time in milliseconds and the number of launches timed. */
enum { IBSN_KT_EVAL = 0,      /* row LSE pass (eval)                                   */
       IBSN_KT_TRIAL,         /* Armijo trial pass                                     */
       IBSN_KT_SPARSIFY,      /* Algorithm 1 pass                                      */
       IBSN_KT_CSC,           /* transpose of the sparsified factor                    */
       IBSN_KT_STOP1,         /* stop test pass 1                                      */
       IBSN_KT_STOP2,         /* stop test pass 2                                      */
       IBSN_KT_CG,            /* one CG solve, host polling included (all iterations)  */
       IBSN_KT_COLRED,        /* column partial reduction                              */
       IBSN_KT_EVAL_MIXED,    /* eval pass in the mixed-precision form                 */
       IBSN_KT_TRIAL_MIXED,   /* Armijo trial pass in the mixed-precision form         */
       IBSN_KT_SPARSIFY_MIXED,/* Algorithm 1 pass in the mixed-precision form          */
       IBSN_KT_N };
typedef struct {
    double ms[IBSN_KT_N];
    int64_t count[IBSN_KT_N];
} ibsn_kernel_times;
int ibsn_kernel_timing(ibsn_ctx *ctx, int enable);
int ibsn_kernel_times_get(ibsn_ctx *ctx, ibsn_kernel_times *out);

/* One record per outer iteration of ibsn_solve (the per-iteration log): counts and times
   are those of this outer iteration alone; the certificate fields are those of its final
   stop pass.  Summed over the records of a solve, the counts and times equal the report's
   totals (t_total aside, which also covers set-up). */
typedef struct {
    int64_t k;                                 /* index of the subproblem (prox centre X^k) */
    int64_t newton, cg, sinkhorn, backtracks, stop_tests, passes, mixed_passes;
    double grad_norm, primal, dual, rel_gap, kkt, dphi, marg_l1;
    double nnz_mean;                           /* mean stored entries of its factors (0: none) */
    double t_eval, t_sparsify, t_cg, t_linesearch, t_stop, t_total;   /* seconds */
    int32_t inner_stopped;                     /* 1: the D_phi test (or (E)IBSN's ||g||) passed */
    int32_t reserved;
} ibsn_iter_record;

/* Solver options; ibsn_default_options() fills the paper's values where it gives
   them (sigma, beta: Algorithm 2 input; Sinkhorn tolerance and mu_k schedule:
   Section 5 "Setup"; 300 outer iterations: Table 1). */
typedef struct {
    double sigma_armijo, beta;           /* 1e-4, 0.8 */
    double sinkhorn_tol;                 /* 1e-3 (Euclidean norm of g) */
    int32_t sinkhorn_maxit;              /* 10000 */
    double mu0, mu_floor;                /* mu_k = max(mu0/(k+1)^2, mu_floor): 1e-4, 1e-11 */
    double gap_tol, marg_tol, kkt_tol;   /* 1e-8 relative gap, 1e-9 ||X^T1-b||_1, 0 = off */
    int32_t max_outer, max_newton, max_backtrack, cg_maxit; /* 300, 1000, 60, 0 = min(n,70) */
    double cg_forcing_max;               /* CG stops at ||r|| <= max(min(0.1, ||g||), */
    int32_t rho_mode;                    /*   cg_rtol_min) ||g||; rho_mode 0: rho =       */
    double cg_rtol_min;                  /*   eta ||g|| / (m n), 1: rho = 0; 1e-6          */
    int32_t stall_limit;                 /* 1: failed D_phi tests (gate passed) that end   */
                                         /*    the inner loop of one outer iteration       */
    int32_t eot;                         /* 1: (E)IBSN of appendix C.4: prox centre 1 1^T,  */
    double eot_tol;                      /*    one subproblem until ||g|| < eot_tol (1e-9) */
    double mixed_switch;                 /* IBSN_PREC_MIXED: Newton steps use the FP32    */
                                         /*   passes while ||g||_2 >= mixed_switch *      */
                                         /*   FLT_EPSILON * ||b||_2 (64), and FP64 after   */
                                         /*   that or after an FP32 line search fails     */
    ibsn_iter_record *trace;             /* host, optional (NULL): the first trace_cap outer */
    int64_t trace_cap;                   /*   iterations' records; ibsn_report.trace_len     */
                                         /*   says how many were written                     */
    int32_t armijo_warm;                 /* 1: each line search starts at                      */
                                         /*   min(1, t_prev / beta), t_prev the step the      */
                                         /*   previous line search accepted; 0: at t = 1. The */
                                         /*   paper leaves the first trial step open; the     */
                                         /*   Armijo condition itself is the same             */
} ibsn_options;

void ibsn_default_options(ibsn_options *opt);

typedef struct {
    int64_t outer, newton, cg, sinkhorn, backtracks, stop_tests, passes;
    double grad_norm, primal, dual, rel_gap, kkt, dphi, marg_l1;
    double t_eval, t_sparsify, t_cg, t_linesearch, t_stop, t_total;  /* seconds */
    double nnz_mean, nnz_last;  /* stored entries of the sparsified factors (mean, last) */
    int64_t mixed_passes;       /* m x n passes run in the FP32 form (IBSN_PREC_MIXED) */
    int64_t trace_len;          /* records written to ibsn_options.trace */
    int32_t status;
} ibsn_report;

/* Full IBSN solve (Algorithm 2 with the practical stop schedule of Section 5).
   gamma_io (n, device): in = warm start (NULL = 0; it is centred), out = final dual.
   r_io (m), s_io (n), k_io (host): optional outer state; when k_io != NULL and
   *k_io > 0 the solve resumes from (k, r, s); on return they hold the final state.
   plan_out (m x n, optional): rounded plan Xhat of the final iterate.
   rep (host, optional).  Stops when the certified relative gap <= gap_tol and
   ||X^T 1 - b||_1 <= marg_tol (marg_tol <= 0: not required), or Delta_kkt <= kkt_tol
   (kkt_tol > 0), or after max_outer outer iterations (returns IBSN_WARN_MAXITER). */
int ibsn_solve(ibsn_ctx *ctx, const ibsn_problem *prob, const ibsn_options *opt,
               double *gamma_io, double *r_io, double *s_io, int64_t *k_io, double *plan_out,
               ibsn_report *rep);

/* Many independent problems (the batched form; the paper solves one problem at a time).
   nctx contexts, each used by one host worker thread of this call, on its own stream:
   the small, launch-latency-bound passes of different problems then overlap on the GPU.
   Problems are taken largest m n first from a shared counter.  For problem i:
   gamma_io[i] (n_i, device; gamma_io or gamma_io[i] may be NULL) is the warm start in and
   the final dual out, reps[i] (optional) its report, status[i] its ibsn_solve return code.
   opt (NULL = defaults) applies to all.  Results do not depend on nctx or on which context
   solved a problem.  Returns IBSN_OK once every problem has been attempted, or
   IBSN_ERR_INVALID_ARG (no problem attempted) for bad arguments, including a context
   passed twice.  The contexts must not be used by other threads during the call. */
int ibsn_solve_batch(ibsn_ctx *const *ctxs, int nctx, int64_t nprob, const ibsn_problem *probs,
                     const ibsn_options *opt, double *const *gamma_io, ibsn_report *reps,
                     int32_t *status);

/* ------------------------------------------------------------------------------------
   Learned warm start for the first subproblem's dual (the paper starts Algorithm 2 from
   gamma^{0,0} = 0; a starting dual only changes where the first subproblem's iteration
   begins, not what it converges to).
   A point-set network: a per-point MLP encoder (3 layers of width 256, ReLU) over the
   sources and the targets, mean pooling per side into a context c = Wc [h_s; h_t] + bc
   (256 values per instance), and a per-target head (2 layers of width 256, ReLU) over the
   target's 8 features f_j whose output is read out against the context, plus a linear
   path from the same features: o_j = z2_j . c + ws . f_j + bo.  The output is centred and
   scaled: gamma_j = scale (o_j - mean o).  Every matrix product of the MLP runs as BF16
   MFMA with FP32 accumulation (operands rounded to BF16 where they enter a product);
   biases, activations, pooling, the linear path, the loss and the Adam update are FP32.
   Features (ibsn_ws_features, 2-D points).  Coordinates are box coordinates: shifted by
   the lower corner of the bounding box of all points and divided by its longer side L.
   u = kappa L^2 is the cost of a unit box distance squared, kappa = sum_{i<K} C_ii /
   sum_{i<K} |x_i - y_i|^2 over the first K = min(m, n, 4096) pairs (the points cost's
   cost_scale for IBSN_COST_POINTS); s = sqrt(mean_j min_i C_ij / u), the typical
   distance from a target to its nearest source in box units; scale = u s.
     fs  (m x 4): (x~_i1, x~_i2, m a_i, 1)          encoder, sources
     fte (n x 4): (y~_j1, y~_j2, n b_j, -1)         encoder, targets
     fth (n x 8): (y~_j1, y~_j2, n b_j, min_i C_ij / mean_j min_i C_ij,
                   (G_k(j) - mean_j G_k) / s, k = 1..4)
   with G_k(j) = sum_i a_i g_k(x~_i, y~_j) - sum_l b_l g_k(y~_l, y~_j),
   g_k(p, q) = log(|p - q|^2 + e_k^2) / 2 summed over the nine mirror images of p in the
   box, e_k = 0.01, 0.02, 0.04, 0.08: the potential of the linearised Monge-Ampere equation
   (its Laplacian is the difference of the two densities, smoothed at e_k, with a
   reflecting boundary), computed with FP32 logarithms and FP64 sums.  FP32 device
   arrays, row-major.
   ------------------------------------------------------------------------------------ */
typedef struct ibsn_ws_model ibsn_ws_model;

/* Number of FP32 parameters (W1 b1 W2 b2 W3 b3 Wf bf Wg bg Wc bc ws bo, weights stored
   inputs x outputs, row-major, concatenated in that order). */
int64_t ibsn_ws_param_count(void);
/* New model on the context's device, weight matrices He-initialised from `seed`; biases,
   the linear path ws and the context map Wc start at zero (the output starts at 0).  Free
   with ibsn_ws_free. */
int ibsn_ws_create(ibsn_ctx *ctx, uint64_t seed, ibsn_ws_model **out);
void ibsn_ws_free(ibsn_ws_model *model);
/* Host copies of the FP32 parameters (count = ibsn_ws_param_count()).  set also resets the
   Adam state and refreshes the BF16 copies.  Synchronise. */
int ibsn_ws_get_params(ibsn_ctx *ctx, const ibsn_ws_model *model, float *host, int64_t count);
int ibsn_ws_set_params(ibsn_ctx *ctx, ibsn_ws_model *model, const float *host, int64_t count);
/* Features of one problem given its 2-D points x (m x 2) and y (n x 2) (device FP64);
   scale_host receives u s (above).  Synchronises. */
int ibsn_ws_features(ibsn_ctx *ctx, const ibsn_problem *prob, const double *x, const double *y,
                     float *fs, float *fte, float *fth, double *scale_host);
/* Raw outputs o (B n, FP32 device) for B instances of m sources and n targets, features
   stacked by instance (fs: B m x 4, fte: B n x 4, fth: B n x 8). */
int ibsn_ws_forward(ibsn_ctx *ctx, ibsn_ws_model *model, int64_t B, int64_t m, int64_t n,
                    const float *fs, const float *fte, const float *fth, float *out);
/* The warm start of one instance: gamma_out (n, FP64 device) = scale (o - mean o). */
int ibsn_ws_predict(ibsn_ctx *ctx, ibsn_ws_model *model, int64_t m, int64_t n, const float *fs,
                    const float *fte, const float *fth, double scale, double *gamma_out);
/* One training step on B instances: loss = mean over instances and targets of
   ((o_j - mean o) - target_j)^2 with target (B n, FP32 device) the centred dual divided
   by its instance's scale; gradients by backpropagation, then one Adam step (beta1 0.9,
   beta2 0.999, eps 1e-8) at learning rate lr (lr = 0: gradients only).  Host out: loss;
   grad_host (optional, parameter count floats) receives the gradient.  Synchronises. */
int ibsn_ws_train_step(ibsn_ctx *ctx, ibsn_ws_model *model, int64_t B, int64_t m, int64_t n,
                       const float *fs, const float *fte, const float *fth, const float *target,
                       float lr, float *loss_host, float *grad_host);

#ifdef __cplusplus
}
#endif

#endif /* IBSN_H */
