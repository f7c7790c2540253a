"""Mixed-precision form (FP32 exponentials and FP32 sparse values, FP64 sums) against the
FP64 oracle, through the C ABI.

Error model, from which every tolerance below follows.  Each exponential of the mixed
passes is exp(x) with x formed in FP64, split as x/ln2 = k + f, f rounded to FP32
(absolute error <= 2^-25, i.e. relative <= 2.3e-8 in 2^f), 2^f from the hardware base-2
exponential (about 1 ulp = 1.2e-7) and 2^k applied exactly.  So each entry carries a
relative error u <= 2.4e-7 (2^-22).  Sums of positive terms keep that bound:
  S_i (row sums)                   relative u
  c_j = sum_i a_i e_ij / S_i       relative 2u          (plan entries likewise)
  lse_i = M_i + log S_i            absolute u
  L = -b^T gamma + eta sum a_i (r_i + lse_i)   absolute eta u
  trial decrease dL: delta_i = log(ratio of two such sums): absolute 2u, and for small
  steps relative 2u of |delta_i| <= t max|Delta| / eta, so |dL error| <= 2u min(eta,
  t max|Delta|)
  sparsify values p / (kept sum), stored as FP32: relative 2u + 2^-24
Tests use twice these bounds.  Below 2^-126 an exponential is an FP32 denormal, whose
absolute error is at most 2^-150 (flushed to 0 below about 2^-149); since a_i <= 1 <= S_i,
plan entries get that as an absolute term.  The instances keep every column sum far
above it.  The sparsity pattern may
differ from the oracle's only where the FP64 value lies within the relative band 4u of rho.
HVP and CG take the factor as stored (FP32 values, widened exactly), so they are compared
with the oracle applied to that exported factor at FP64 tolerances.  The full solve
switches to FP64 passes near convergence and is held to the FP64 bar.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2603_07156_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U = 2.0 ** -22


@pytest.fixture(scope="module")
def ib():
    from paper_2603_07156_amd import ibsn
    return ibsn


@pytest.fixture(scope="module")
def ctx(ib):
    return ib.Context(0)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def mproblem(ib, inst, C=None):
    C = inst.C if C is None else C
    return ib.Problem(dev(C), dev(inst.a), dev(inst.b), inst.eta, precision=ib.PREC_MIXED)


def outer_state(inst, k):
    if k == 0:
        return np.log(inst.a), np.log(inst.b), 0, W.random_dual(inst.n, 17, 0.02)
    opt = orc.default_options(max_outer=k, gap_tol=0.0, marg_tol=0.0)
    res = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=opt)
    return res["r"], res["s"], res["k"], res["gamma"] + W.random_dual(inst.n, 3, 1e-4)


def center(ib, inst, r, s, k, gamma, C=None):
    q = orc.center_quantum(inst.C if C is None else C, s, gamma, inst.eta, k)
    return ib.Center(k, dev(r), dev(s), q), q


def lo_split(C):
    """Whether the library carries the low parts of the potentials for this cost: not for
    FP32 costs wider than 12288 columns, whose tiles have no LDS left for them."""
    return not (C.dtype == np.float32 and C.shape[1] > 12288)


def check_eval_mixed(ib, ctx, inst, r, s, k, gamma, C=None, want_plan=True):
    Cc = inst.C if C is None else C
    pr = mproblem(ib, inst, Cc)
    ctr, q = center(ib, inst, r, s, k, gamma, Cc)
    gv = ib.subproblem_eval(ctx, pr, ctr, dev(gamma), want_obj=True, want_plan=want_plan)
    ov = orc.eval_pass(Cc, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=k, want_plan=want_plan,
                       q=q, split=lo_split(Cc))
    # the row maxima involve no exponential: identical bits
    np.testing.assert_array_equal(host(gv["M"]), ov.M)
    np.testing.assert_allclose(host(gv["S"]), ov.S, rtol=2 * U)
    np.testing.assert_allclose(host(gv["lse"]), ov.lse, rtol=0, atol=2 * U)
    c = host(gv["c"])
    assert ov.c.min() > 1e-30
    np.testing.assert_allclose(c, ov.c, rtol=4 * U)
    np.testing.assert_allclose(host(gv["g"]), ov.g, rtol=0, atol=4 * U * ov.c.max())
    assert abs(gv["L"] - ov.L) <= 2 * U * inst.eta + 1e-13 * abs(ov.L)
    if want_plan:
        np.testing.assert_allclose(host(gv["plan"]), ov.plan, rtol=4 * U, atol=2.0 ** -148)
    # on instances with many entries per row the error shows the FP32 level: the mixed
    # form ran
    if Cc.shape[1] >= 64:
        assert np.abs(host(gv["S"]) / ov.S - 1).max() > 1e-13
    return gv, ov


@pytest.mark.parametrize("m,n", [(1, 1), (3, 2), (41, 65), (300, 257), (70, 513), (33, 2047),
                                 (17, 2049), (8, 8191), (5, 10240)])
def test_eval_mixed_shapes(ib, ctx, m, n):
    inst = W.gmm_points(n, 5, m=m)
    r, s, k, gamma = outer_state(inst, 0)
    if n > 1:
        check_eval_mixed(ib, ctx, inst, r, s, k, gamma)
    else:
        # one column: P = 1 exactly on both sides
        pr = mproblem(ib, inst)
        ctr, q = center(ib, inst, r, s, k, gamma)
        gv = ib.subproblem_eval(ctx, pr, ctr, dev(gamma), want_obj=True)
        np.testing.assert_allclose(host(gv["c"]), [1.0], rtol=1e-15)


@pytest.mark.parametrize("k", [4, 25])
def test_eval_mixed_outer_states(ib, ctx, k):
    """Large sigma = (k+1)/eta: the FP64 argument keeps the FP32 exponential accurate."""
    inst = W.uniform_points(300, 1, m=260)
    r, s, kk, gamma = outer_state(inst, k)
    check_eval_mixed(ib, ctx, inst, r, s, kk, gamma)


def test_eval_mixed_fp32_cost(ib, ctx):
    inst = W.gmm_points(1500, 9, m=200)
    C32 = inst.C.astype(np.float32)
    r, s, k, gamma = outer_state(inst, 0)
    check_eval_mixed(ib, ctx, inst, r, s, k, gamma, C=C32)


def test_eval_mixed_full_size_10k(ib, ctx):
    """10^4 x 10^4 in the benchmark's launch configuration."""
    inst = W.uniform_points(10000, 1000)
    r, s, k, gamma = np.log(inst.a), np.log(inst.b), 0, W.random_dual(10000, 2, 0.01)
    check_eval_mixed(ib, ctx, inst, r, s, k, gamma, want_plan=False)


@pytest.mark.parametrize("t", [1.0, 1e-3, 1e-9])
def test_trial_mixed(ib, ctx, t):
    inst = W.gmm_points(513, 12, m=301)
    r, s, kk, gamma = outer_state(inst, 6)
    ctr, q = center(ib, inst, r, s, kk, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=kk, q=q)
    Delta = W.random_dual(513, 44, 0.02)
    pr = mproblem(ib, inst)
    gt = ib.trial(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(Delta), t)
    dL, Mn, Sn, cn, gn = orc.trial_pass(inst.C, inst.a, inst.b, inst.eta, gamma, ev.M, Delta, t,
                                        s=s, k=kk, q=q)
    bound = 4 * U * min(inst.eta, t * np.abs(Delta).max())
    assert abs(gt["dL"] - dL) <= bound + 1e-12 * abs(dL), (gt["dL"], dL, bound)
    np.testing.assert_allclose(host(gt["M"]) + np.log(host(gt["S"])), Mn + np.log(Sn), rtol=0,
                               atol=4 * U)
    np.testing.assert_allclose(host(gt["c"]), cn, rtol=6 * U)
    np.testing.assert_allclose(host(gt["g"]), gn, rtol=0, atol=6 * U * np.abs(cn).max())


@pytest.mark.parametrize("scale", [0.04, 0.1])
def test_trial_mixed_large_step(ib, ctx, scale):
    """Steps with max tau = t Delta / eta in (89, 500]: the small form keeps q e^tau unshifted
    there, which would overflow an FP32 value (e^89 > FLT_MAX), so the mixed trial hands
    steps with max tau > 80 to the FP64 pass.  All outputs finite and within the error model
    against the FP64 oracle."""
    inst = W.gmm_points(300, 2, m=200)
    inst = W.Instance(inst.C, inst.a, inst.b, 1e-3, "large_step")
    r, s, k, gamma = np.log(inst.a), np.log(inst.b), 0, np.zeros(300)
    ctr, q = center(ib, inst, r, s, 0, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, q=q)
    Delta = W.random_dual(300, 7, scale)
    tau_max = np.abs(Delta).max() / inst.eta
    assert 89 < Delta.max() / inst.eta <= 500, Delta.max() / inst.eta
    pr = mproblem(ib, inst)
    gt = ib.trial(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(Delta), 1.0)
    dL, Mn, Sn, cn, gn = orc.trial_pass(inst.C, inst.a, inst.b, inst.eta, gamma, ev.M, Delta, 1.0,
                                        s=s, q=q)
    for key in ("M", "S", "c", "g"):
        assert torch.isfinite(gt[key]).all(), key
    assert np.isfinite(gt["dL"])
    bound = 4 * U * min(inst.eta, tau_max * inst.eta)
    assert abs(gt["dL"] - dL) <= bound + 1e-12 * abs(dL), (gt["dL"], dL, bound)
    np.testing.assert_allclose(host(gt["M"]) + np.log(host(gt["S"])), Mn + np.log(Sn), rtol=0,
                               atol=4 * U)
    # The small form's q e^tau = q + q expm1(tau) cancels for tau << 0 (both sides): columns
    # whose steps are very negative carry an absolute error at the level of the unstepped
    # column sum, far below max c.
    np.testing.assert_allclose(host(gt["c"]), cn, rtol=6 * U, atol=1e-14 * np.abs(cn).max())
    np.testing.assert_allclose(host(gt["g"]), gn, rtol=0, atol=6 * U * np.abs(cn).max())


def exported_csr(gcsr, m, n):
    row_ptr, col, val, d = (host(x) for x in gcsr.export())
    return orc.CSR(m, n, row_ptr.astype(np.int64), col.astype(np.int32), val, d, gcsr.istar)


@pytest.mark.parametrize("rho_rule", ["zero", "paper", "1e-5"])
def test_sparsify_hvp_cg_mixed(ib, ctx, rho_rule):
    m, n = 420, 600
    inst = W.gmm_points(n, 8, m=m)
    r, s, kk, gamma = outer_state(inst, 5)
    ctr, q = center(ib, inst, r, s, kk, gamma)
    ev = orc.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, r=r, s=s, k=kk, want_plan=True,
                       q=q)
    P = ev.plan / inst.a[:, None]
    rho = {"zero": 0.0, "paper": inst.eta * np.linalg.norm(ev.g) / P.size, "1e-5": 1e-5}[rho_rule]
    pr = mproblem(ib, inst)
    gcsr = ib.sparsify(ctx, pr, ctr, dev(gamma), dev(ev.M), dev(ev.S), rho)
    ocsr = orc.sparsify(inst.C, inst.a, inst.eta, gamma, ev.M, ev.S, rho, s=s, k=kk, q=q)
    g = exported_csr(gcsr, m, n)
    assert g.istar == ocsr.istar == int(np.argmax(inst.a))
    assert int(g.row_ptr[-1]) == gcsr.nnz
    # values are FP32 numbers
    assert np.array_equal(g.val.astype(np.float32).astype(np.float64), g.val)
    differing = 0
    for i in range(m):
        gc = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
        oc = ocsr.col[ocsr.row_ptr[i]:ocsr.row_ptr[i + 1]]
        assert np.all(np.diff(gc) > 0)
        if np.array_equal(gc, oc):
            np.testing.assert_allclose(g.val[g.row_ptr[i]:g.row_ptr[i + 1]],
                                       ocsr.val[ocsr.row_ptr[i]:ocsr.row_ptr[i + 1]],
                                       rtol=6 * U, atol=2.0 ** -148)
        else:
            differing += 1
            diff = np.setxor1d(gc, oc)
            assert np.all(np.abs(P[i, diff] - rho) <= 4 * U * rho), (i, diff)
    # d = P~^T (a o P~ 1) for the stored factor P~ (FP64 sums); P~ 1 = 1 to FP32 rounding
    rows = np.repeat(np.arange(m), np.diff(g.row_ptr))
    rsum = np.zeros(m)
    np.add.at(rsum, rows, g.val)
    assert np.abs(rsum[np.diff(g.row_ptr) > 0] - 1).max() <= 2e-6
    dd = np.zeros(n)
    np.add.at(dd, g.col, (inst.a * rsum)[rows] * g.val)
    np.testing.assert_allclose(g.d, dd, rtol=1e-12)
    if differing == 0:
        np.testing.assert_allclose(g.d, ocsr.d, rtol=6 * U)
    # HVP and CG on the stored factor: FP64 arithmetic on identical values
    for shift in (0.0, 1e-3):
        v = W.random_dual(n, 21, 1.0)
        yg = host(ib.hvp(ctx, gcsr, pr.a, inst.eta, shift, dev(v)))
        yo = orc.hvp(g, inst.a, inst.eta, shift, v)
        np.testing.assert_allclose(yg, yo, rtol=1e-12, atol=1e-12 * np.abs(yo).max())
    ones = torch.ones(n, dtype=torch.float64, device="cuda")
    h1 = host(ib.hvp(ctx, gcsr, pr.a, inst.eta, 0.0, ones))
    assert np.abs(h1).max() <= 1e-12 / inst.eta   # Theorem 3.2 on the stored factor
    gn = np.linalg.norm(ev.g)
    shift = max(gn, 1e-2)
    tol = 1e-12 * gn
    xg, itg = ib.cg(ctx, gcsr, pr.a, inst.eta, shift, dev(-ev.g), tol, 500)
    xo, ito = orc.cg(g, inst.a, inst.eta, shift, -ev.g, tol, 500)
    assert itg < 500 and ito < 500
    np.testing.assert_allclose(host(xg), xo, rtol=0, atol=1e-9 * np.abs(xo).max())
    gcsr.free()


def test_solve_mixed_n64_exact(ib, ctx):
    """The mixed form reaches the exact optimum (the final steps run in FP64)."""
    from scipy.optimize import linear_sum_assignment
    inst = W.uniform_points(64, 0)
    rr, cc = linear_sum_assignment(inst.C)
    fstar = inst.C[rr, cc].sum() / 64
    pr = mproblem(ib, inst)
    opt = ib.default_options(max_outer=20000, gap_tol=1e-8, marg_tol=0.0)
    res = ib.solve(ctx, pr, opt, want_plan=True)
    rep = res["report"]
    assert res["status"] == 0, rep
    assert rep["mixed_passes"] > 0
    assert rep["rel_gap"] <= 1e-8
    assert rep["dual"] <= fstar * (1 + 1e-13) and rep["primal"] >= fstar * (1 - 1e-13)
    X = host(res["plan"])
    np.testing.assert_allclose(X.sum(1), inst.a, atol=1e-15 * 64, rtol=0)
    np.testing.assert_allclose(X.sum(0), inst.b, atol=1e-15 * 64, rtol=0)


def test_solve_mixed_general_weights_vs_oracle(ib, ctx):
    """Objective and plan of the mixed solve against the FP64 oracle and HiGHS, both
    solves run to a certified relative gap of 1e-10: the objectives then agree to 1e-10
    relative (each lies in [f*, f*(1 + 1e-10)]) and the plans to 1e-9 per entry."""
    from scipy.optimize import linprog
    m, n = 24, 20
    inst = W.gmm_points(n, 101, m=m)
    A_eq = np.zeros((m + n, m * n))
    for i in range(m):
        A_eq[i, i * n:(i + 1) * n] = 1.0
    for j in range(n):
        A_eq[m + j, j::n] = 1.0
    fstar = linprog(inst.C.ravel(), A_eq=A_eq, b_eq=np.concatenate([inst.a, inst.b]),
                    bounds=(0, None), method="highs").fun
    opt_kw = dict(max_outer=20000, gap_tol=1e-10, marg_tol=0.0)
    pr = mproblem(ib, inst)
    res = ib.solve(ctx, pr, ib.default_options(**opt_kw), want_plan=True)
    rep = res["report"]
    assert res["status"] == 0, rep
    assert rep["mixed_passes"] > 0
    o = orc.solve(inst.C, inst.a, inst.b, inst.eta, options=orc.default_options(**opt_kw),
                  want_plan=True)
    assert o["status"] == 0
    assert abs(rep["primal"] - o["report"]["primal"]) <= 1e-10 * abs(o["report"]["primal"])
    assert abs(rep["primal"] - fstar) <= 1e-8 * fstar
    np.testing.assert_allclose(host(res["plan"]), o["plan"], rtol=0, atol=1e-9)


def test_mixed_switch_zero_runs_mixed_to_the_end(ib, ctx):
    """mixed_switch = 0 keeps the FP32 passes for every Newton step whose line search
    succeeds; the stop test still runs on FP64 states, so the certificate holds."""
    inst = W.uniform_points(64, 0)
    pr = mproblem(ib, inst)
    opt = ib.default_options(max_outer=200, gap_tol=0.0, marg_tol=0.0, mixed_switch=0.0)
    res = ib.solve(ctx, pr, opt)
    rep = res["report"]
    assert rep["mixed_passes"] > 0
    assert rep["primal"] >= rep["dual"] - 1e-14


def test_cfg3_full_size_fp32_cost(ib, ctx):
    """20000 x 20000, 3-D unit-cube points vs an 8-component mixture, cost stored FP32
    (1.6 GB): the mixed eval against the oracle on the same (widened) cost, and the FP64
    stop pass, whose staged n-vector plus static LDS is the largest request of the dense
    passes (it must fit the 160 KB per workgroup)."""
    inst = W.cube_vs_gmm(20000, 200, cost_dtype=np.float32)
    r, s, k, gamma = np.log(inst.a), np.log(inst.b), 0, W.random_dual(20000, 4, 0.01)
    gv, ov = check_eval_mixed(ib, ctx, inst, r, s, k, gamma, want_plan=False)
    pr = ib.Problem(dev(inst.C), dev(inst.a), dev(inst.b), inst.eta)
    ctr, q = center(ib, inst, r, s, k, gamma)
    gs = ib.stop(ctx, pr, ctr, dev(gamma), dev(ov.M), dev(ov.S))
    os_ = orc.stop_pass(inst.C, inst.a, inst.b, inst.eta, gamma, ov.M, ov.S, s=s, k=k, q=q,
                        split=lo_split(inst.C))
    # 4e8 terms: both sides sum per row (GPU: per thread) before the totals; each is within
    # a few 1e-15 of an exactly rounded sum
    for key in ("primal", "cx"):
        assert abs(gs[key] - os_[key]) <= 1e-12 * abs(os_[key]), (key, gs[key], os_[key])
