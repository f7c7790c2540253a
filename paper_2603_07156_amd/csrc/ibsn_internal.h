// ibsn_internal.h -- launchers shared by the HIP translation units of libibsn.so.
// Not installed; the public ABI is include/ibsn.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibsn {

// Work split of the dense row passes: `grid` workgroups, workgroup g owns rows
// [m*g/grid, m*(g+1)/grid), and writes one n-long column partial row.
struct RowPlan {
    int nt;              // threads per workgroup (eval, stop pass 1)
    int q;               // vector slots per thread (row held as q*vec values per thread)
    int qf;              // leading slabs that lie inside the row for every thread
    int nt_h, q_h, qf_h; // the same for trial and sparsify
    int vec;             // elements per vector load (2 for FP64 cost, 4 for FP32)
    int grid;            // number of workgroups (all passes)
    // rows split into nb column blocks of bw columns (the last one narrower); the tile
    // fields then describe a block of bw columns.  nb = 1: whole rows (bw = n).
    int nb = 1;
    int64_t bw = 0;
};

// Choose the register tile for a row of n entries; returns false if n is too large.
bool plan_rows(int64_t m, int64_t n, int cost_kind, int num_cus, RowPlan *plan);
// the same plan with the heavy tile (trial, sparsify) as the tile
RowPlan heavy_plan(const RowPlan &p);
// Compiled light (eval, stop) or heavy (trial, sparsify) tiles that can hold a row of n
// entries with their first QF slabs inside it: up to cap rows {NT, Q, QF}; returns the count.
int tile_candidates(int64_t n, int cost_kind, bool heavy, int (*out)[3], int cap);

// Two-level potentials: w_j = wh_j + wl_j with wh on the grid of spacing q and wl the
// remainder (|wl| <= q/2 plus rounding).  The dense passes stage wl as FP32 after the n
// doubles they stage; a tile spanning more than LO_MAX_COLS columns (FP32 cost beyond
// that many columns) has no LDS left for it, and there the host keeps wl = 0 (potentials
// and steps rounded to the grid).
constexpr int LO_MAX_COLS = 12288;
__host__ __device__ constexpr bool lo_tile(int nt, int q, int vec) { return nt * q * vec <= LO_MAX_COLS; }

struct DenseArgs {
    const void *C;            // the cost, or x (m x pdim) for points
    int64_t ldc;
    const double *py;         // points: y (n x pdim)
    double pscale;            // points: cost scale
    int pdim;                 // points: 2 or 3
    int64_t m, n;
    int cost_kind;
    double sigma;           // (k+1)/eta
    double q;               // grid spacing of the potentials (power of two)
    const double *w;        // n: high part of the potentials, on the grid
    const double *wlo;      // n: low part (zero where the tile has no room for it)
    const double *a;        // m
    int mixed;              // 1: FP32 exponentials and FP32 sparse values (eval, trial,
                            // sparsify); sums, shifts and row state stay FP64
    // column block of a split row (C, py, w and wlo then point at the block's first column
    // and n is the block's width): row pitch of the m x n outputs (plan, rounded plan,
    // sparse slots) and the block's first column in them
    int64_t ldo;
    int64_t coff;
};

// ---- eval (fresh row LSE) ------------------------------------------------------
// Writes M (grid-rounded row maxima), S (and lse if non-null), plan (optional),
// colpart[grid][n] = column partials of a_i P_ij,
// rowpart[grid] = sum_i a_i ((r_i + M_i) + log S_i).
// Null colpart / rowpart / M: not written.  Mfull, fscale: the second launch of a column
// block of a split row (column partials and plan from the whole row's shift and a_i / S_i).
hipError_t launch_eval(const RowPlan &p, const DenseArgs &d, const double *r, double *M, double *S,
                       double *lse, double *plan, double *colpart, double *rowpart,
                       hipStream_t st, const double *Mfull = nullptr,
                       const double *fscale = nullptr);

// ---- column log-sum-exp (Sinkhorn step in the log domain) -----------------------
// lc_j = log sum_i a_i exp(x_ij) / S_i from the row state (M, S) at w (lo: with the low
// parts); RB row blocks (collse_row_blocks), pmax and psum RB*n doubles each.
constexpr int COLLSE_MAX_RB = 64;
int collse_row_blocks(int64_t m, int64_t n, int max_rb);
hipError_t launch_collse(const DenseArgs &d, int lo, const double *M, const double *S, int RB,
                         double *pmax, double *psum, double *lc, hipStream_t st);

// ---- Armijo trial --------------------------------------------------------------
// big = 0: colv = expm1(tau) (small-step form); big = 1: colv = exp(tau - tau_max).
// Writes M_new, S_new, colpart (a_i P'_ij), rowpart = sum a_i delta_i.
// Launches both forms; each returns at once unless scal[SC_BIG] selects it, so the
// choice needs no host round trip.  tau_shift is read from scal[SC_TAUSHIFT].
// Null colpart / rowpart / M_new: not written.  rowred (4 m-vectors: Z, A, B, max q e^tau)
// and fscale (a_i / Z_i of the whole row): the two launches of a column block of a split row.
hipError_t launch_trial(const RowPlan &p, const DenseArgs &d, const double *M, const double *colv,
                        const double *scal, double *M_new, double *S_new, double *colpart,
                        double *rowpart, hipStream_t st, double *rowred = nullptr,
                        const double *fscale = nullptr);

// ---- sparsify (Algorithm 1) ----------------------------------------------------
// Slotted CSR: row i's kept entries at [i*n, i*n + len_i), columns ascending.
// colpart = column partials of a_i [P_rho]_ij (for d = P_rho^T a).
// Null colpart: not written.  ksum: a column block of a split row (see k_sparsify).
hipError_t launch_sparsify(const RowPlan &p, const DenseArgs &d, const double *M, const double *S,
                           double rho, const int *istar, int32_t *col, void *val, int32_t *len,
                           double *colpart, hipStream_t st, double *ksum = nullptr);

// ---- stop test, pass 1 (Algorithm 3 rows/columns) -------------------------------
// z_i = min(a_i / sum_j X_ij, 1); colpart  = column partials of X;
// colpart2 = column partials of z_i X_ij; rowpart = sum_i (sum_j X_ij - a_i)^2.
// Null outputs are not written.  rsum (block row sums of X) and zin (z given): the two
// launches of a column block of a split row.
hipError_t launch_stop1(const RowPlan &p, const DenseArgs &d, const double *M, const double *S,
                        double *z, double *colpart, double *colpart2, double *rowpart,
                        hipStream_t st, double *rsum = nullptr, const double *zin = nullptr);

// ---- stop test, pass 2 (rounded plan, D_phi, certificate) -----------------------
struct Stop2Vec {
    const double *gamma, *psi, *y, *ec, *z;   // n, n, n, n, m
    double *er_row, *zg_row;                  // m, m: e_r,i and min_j (C_ij - gamma_j)
    const double *er1;                        // ||e_r||_1 (device scalar)
};
// rowpart[grid * 10]: per-workgroup sums (see STOP2_* slots).
enum { STOP2_DPHI = 0, STOP2_CXH, STOP2_AZG, STOP2_AZP, STOP2_CX, STOP2_XU, STOP2_XHMIN,
       STOP2_XF, STOP2_CF, STOP2_NEG, STOP2_NSLOT };
// which: 1 pass 2a, 2 pass 2b, 3 both.  rowred (three m-vectors): pass 2a of a column block
// of a split row writes its per-row partials there instead of e_r, zg and the sums.
hipError_t launch_stop2(const RowPlan &p, const DenseArgs &d, const double *M, const double *S,
                        const Stop2Vec &v, double *xhat, double *rowpart, hipStream_t st,
                        int which = 3, double *rowred = nullptr);

// ---- column reduction ----------------------------------------------------------
// out_j = sum_g part[g][j] in a fixed order; if sub != null, out2_j = out_j - sub_j.
hipError_t launch_colreduce(const double *part, int G, int64_t n, double *out, const double *sub,
                            double *out2, hipStream_t st);

// ---- rows split into column blocks (dense_wide.hip) -------------------------------
// Per-block row arrays: nb consecutive m-vectors.  G: workgroups, each joining a range of
// rows and writing one partial sum per row range.
// eval: M, S, lse (optional) of the whole row, f_i = a_i / S_i, rowpart[G] = objective
// terms (r given).
hipError_t launch_wide_eval_rows(int64_t m, int nb, const double *Mb, const double *Sb,
                                 const double *a, const double *r, double *M, double *S,
                                 double *lse, double *f, double *rowpart, int G, hipStream_t st);
// trial: rr = per block 4 m-vectors (Z, A, B, max q e^tau); new row state, f_i = a_i / Z_i,
// rowpart[G] = sum a_i delta_i
hipError_t launch_wide_trial_rows(int64_t m, int nb, const double *rr, const double *a,
                                  const double *M, const double *scal, double qg, double *Mn,
                                  double *Sn, double *f, double *rowpart, int G, hipStream_t st);
// sparsify: join the blocks' segments of each row (block b at column offset b bw of the
// row's slot, lenb entries, kept sum ksb), normalise, write len and the row weights u of d
hipError_t launch_wide_join(int64_t m, int64_t n, int nb, int64_t bw, const int32_t *lenb,
                            const double *ksb, const double *a, const int *istar, int32_t *col,
                            void *val, int f32, int32_t *len, double *u, hipStream_t st);
struct CsrView;
// d_j = sum_i u_i P_ij from the transpose and the dense row
hipError_t launch_wide_d(const CsrView &c, const double *u, double *d, hipStream_t st);
// stop pass 1: z from the blocks' row sums of X; rowpart[G] = sum (X1 - a)_i^2
hipError_t launch_wide_stop1_rows(int64_t m, int nb, const double *rsb, const double *a, double *z,
                                  double *rowpart, int G, hipStream_t st);
// stop pass 2a: rr = per block 3 m-vectors (sum X y, min C - gamma, min C - psi); e_r, zg,
// and the AZG / AZP slots of rowpart[G * STOP2_NSLOT]
hipError_t launch_wide_stop2a_rows(int64_t m, int nb, const double *rr, const double *a,
                                   const double *z, double *er, double *zg, double *rowpart,
                                   int G, hipStream_t st);

// ---- small vector / scalar kernels ----------------------------------------------
// w = s + gamma/eta as a two-level potential (w on the grid of spacing q, wlo the rest);
// split = 0: w = grid(s + gamma/eta), wlo = 0.  gamma may be null.
hipError_t launch_make_w(const double *s, const double *gamma, double q, double eta, int64_t n,
                         int split, double *w, double *wlo, hipStream_t st);
// out[0] = sum_i x_i (fixed order) for up to n values, single workgroup
hipError_t launch_sum(const double *x, int64_t n, double *out, hipStream_t st);
// out[0] = sum_i x_i * y_i (fixed order), single workgroup
hipError_t launch_dot(const double *x, const double *y, int64_t n, double *out, hipStream_t st);

// Sparse structures -------------------------------------------------------------
struct CscWork {
    int64_t *colptr;     // n+1
    int64_t *colcnt;     // n
    int32_t *rowidx;     // capacity m*n
    void *cval;          // capacity m*n values (FP64, or FP32 for a mixed-precision factor)
    uint32_t *mask;      // csc_row_blocks(m) * n: rows of a 32-row block keeping column j
    int32_t *off;        // csc_row_blocks(m) * n: exclusive scan of the mask popcounts
    int lpc;             // lanes per row of the fill (16 or 64)
    int fill = 0;        // CSC_FILL_AUTO, CSC_FILL_ENTRY or CSC_FILL_BLOCK
};
// the transpose's fill: chosen on the device from the stored entries (from
// CSC_BLOCK_MIN_DENSITY m n on by row block), or forced
enum { CSC_FILL_AUTO = 0, CSC_FILL_ENTRY = 1, CSC_FILL_BLOCK = 2 };
constexpr double CSC_BLOCK_MIN_DENSITY = 1.0 / 32.0;
// number of 32-row blocks of the transpose
int csc_row_blocks(int64_t m);
// transpose of the slotted rows without the dense row istar (device scalar)
hipError_t launch_build_csc(int64_t m, int64_t n, const int32_t *col, const void *val, int f32,
                            const int32_t *len, const int *istar, CscWork &w, int64_t *nnz_dev,
                            hipStream_t st);

// Device view of a sparsified factor: slotted rows plus the CSC of the rows != istar.
struct CsrView {
    int64_t m, n;
    const int32_t *col;
    const void *val;          // FP64, or FP32 when f32
    const int32_t *len;
    const int *istar;         // device scalar
    const int64_t *colptr;
    const int32_t *rowidx;
    const void *cval;         // same type as val
    const double *d;          // column sums d_j of the sparsified plan (FP64)
    int f32;
};

// Launch shape of the two gathers of an HVP (and of the CG vector kernels).
enum { CG_MAX_STAR = 64, CG_MAX_COLGROUPS = 2048, CG_MAX_UPDGROUPS = 128 };
struct GatherPlan {
    bool lds;                 // gathered vectors staged in LDS (persistent 1024-thread grid)
    int lpc_row, lpc_col;     // lanes per row / per column
    int row_blocks;           // workgroups of the sparse rows
    int nstar, star_chunk;    // dense-row chunks (extra workgroups) and their width
    int col_blocks;           // column-gather workgroups (grid-stride)
    int upd_blocks;           // CG update workgroups
    bool fused;               // two-kernel CG iterations (LDS path, n <= CG_FUSED_MAX_N)
};
// largest n for which the CG vector update is folded into the next row gather
constexpr int64_t CG_FUSED_MAX_N = 4096;
GatherPlan gather_plan(int64_t m, int64_t n, int64_t nnz, int64_t istar, int num_cus,
                       size_t max_lds);

// y = (H_rho + shift I) v; au (m) and star_part (CG_MAX_STAR) are scratch
hipError_t launch_hvp(const GatherPlan &g, const CsrView &c, const double *a, double eta,
                      double shift, const double *v, double *y, double *au, double *star_part,
                      hipStream_t st);

// CG on the device.  Scalars (CG_* slots) are double-buffered by iteration parity.
struct CgState {
    double *x, *r, *p, *Ap, *au;   // n, n, n, n, m
    double *r2;                    // n: second residual buffer (two-kernel CG, by parity)
    double *star_part;             // CG_MAX_STAR
    double *pap_part;              // CG_MAX_COLGROUPS
    double *rr_part;               // CG_MAX_UPDGROUPS
    double *scal;                  // CG_NSLOT
};
// CG_FIN: the iteration at which the single-workgroup state kernel (two-kernel form)
// finished CG and applied the last update itself; -1 otherwise.
enum {
    CG_TOL = 0, CG_MAXIT, CG_BRK, CG_RR0, CG_RR1, CG_BETA0, CG_BETA1, CG_DONE0, CG_DONE1,
    CG_IT0, CG_IT1, CG_FIN, CG_NSLOT
};
hipError_t launch_cg_init(int64_t n, const double *rhs, double tol, int maxit, CgState &s,
                          hipStream_t st);
// iteration `it` (0-based): three kernels; a no-op once CG has finished
hipError_t launch_cg_iteration(const GatherPlan &g, const CsrView &c, const double *a, double eta,
                               double shift, CgState &s, int it, hipStream_t st);
// writes the state after `it` iterations to slot it&1 (rr, done, iteration count)
hipError_t launch_cg_check(const GatherPlan &g, CgState &s, int it, int64_t n, hipStream_t st);

// CG in one cooperative launch (cg_persistent.hip): `blocks` resident workgroups of 256
// threads, `lanes` lanes per row and per column.  pp: CG_PERSIST_SCRATCH(blocks) doubles
// of partial sums and barrier state.  Results in s.x and s.scal (slot 0: CG_IT0, CG_RR0,
// CG_DONE0, CG_BRK); the error flag (a barrier wait that timed out) is the unsigned at
// pp + 5 blocks + 1.
constexpr int CG_PERSIST_MAX_GRID = 1024;
#define CG_PERSIST_SCRATCH(blocks) (5 * (int64_t)(blocks) + 1)
struct CgPersistPlan {
    int blocks, lanes;
};
CgPersistPlan cg_persist_plan(int64_t m, int64_t n, int64_t nnz, int64_t istar, int num_cus,
                              int blocks);
hipError_t launch_cg_persist(const CgPersistPlan &pl, const CsrView &c, const double *a,
                             double eta, double shift, const double *rhs, double tol, int maxit,
                             CgState &s, double *pp, hipStream_t st);

// CG in one workgroup of 1024 threads (cg_single.hip): p and u in LDS ((m + n) doubles),
// at most CG_SINGLE_MAX_COLS_PER_THREAD columns per thread.  Results as launch_cg_persist.
constexpr int CG_SINGLE_MAX_COLS_PER_THREAD = 10;
// The automatic choice takes the one-workgroup CG for factors of at most
// CG_SINGLE_ENTRIES_PER_LINE max(m, n) entries with m, n <= CG_SINGLE_MAX_DIM.  Each thread
// walks the entries of its rows (and columns) one after another, so the iteration grows
// with the entries per thread: measured per iteration at 2000^2 with 2 entries per row
// 8.1 us against 10.7 (one cooperative launch) and 17.0 (three launches), at 10^4 45 us
// against 15.3 and 15.5; on the early, denser factors of the batched workload it was
// several times slower than the other forms.
constexpr double CG_SINGLE_ENTRIES_PER_LINE = 3.0;
constexpr int64_t CG_SINGLE_MAX_DIM = 4096;
size_t cg_single_lds(int64_t m, int64_t n);
bool cg_single_fits(int64_t m, int64_t n, size_t max_lds);
hipError_t launch_cg_single(const CsrView &c, const double *a, double eta, double shift,
                            const double *rhs, double tol, int maxit, CgState &s,
                            hipStream_t st);

// CG with one grid barrier per iteration (cg_pipe.hip): M = P'^T diag(a) P' built per solve
// (count and scan, then fill; mptr n + 1, its total at mptr[n]), then the pipelined
// recurrences in one cooperative launch of `blocks` workgroups of 256 threads, `lanes`
// (4 or 16) lanes per row of M.  w: 2 n doubles; pp: CG_PIPE_SCRATCH(blocks) doubles of
// partial sums and barrier state (error flag: the unsigned at pp + 6 blocks + 1).
#define CG_PIPE_SCRATCH(blocks) (6 * (int64_t)(blocks) + 1)
// out[0] = sum over rows != istar of len_i^2 (the number of entries of M)
hipError_t launch_len_sq(int64_t m, const int32_t *len, const int *istar, int64_t *out,
                         hipStream_t st);
hipError_t launch_m_count(const CsrView &c, int64_t *cnt, int64_t *mptr, hipStream_t st);
hipError_t launch_m_fill(const CsrView &c, const double *a, const int64_t *mptr, int32_t *mcol,
                         double *mval, hipStream_t st);
int cg_pipe_lanes(int64_t n, int64_t total);
// rows of M per lane group for a grid; at most CG_PIPE_MAX_ROWS (held in registers)
constexpr int CG_PIPE_MAX_ROWS = 8;
int cg_pipe_rows(int64_t n, int blocks, int lanes);
hipError_t launch_cg_pipe(int blocks, int lanes, const CsrView &c, int64_t istar, const double *a,
                          const int64_t *mptr, const int32_t *mcol, const double *mval,
                          const double *rhs, double eta, double shift, double tol, int maxit,
                          CgState &s, double *w, double *pp, hipStream_t st);
// The automatic choice takes the one-barrier form when M has at most CG_PIPE_MAX_RATIO times
// the factor's entries (plus n).
constexpr double CG_PIPE_MAX_RATIO = 4.0;

// export slotted CSR to standard CSR
hipError_t launch_export_csr(int64_t m, int64_t n, const int32_t *col, const void *val, int f32,
                             const int32_t *len, int64_t *row_ptr, int32_t *ocol, double *oval,
                             int64_t cap, hipStream_t st);

// ---- context access for the other translation units of the C ABI -----------------
// (ibsn_ctx is defined in ibsn_api.hip)
}  // namespace ibsn
struct ibsn_ctx;
namespace ibsn {
hipStream_t ctx_stream(const ibsn_ctx *ctx);
int ctx_device(const ibsn_ctx *ctx);
// record the message on ctx and return code (as every entry point does on error)
int ctx_fail(ibsn_ctx *ctx, int code, const char *msg);
}  // namespace ibsn
